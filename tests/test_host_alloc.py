"""Host logic of the serving scheduler: the arena range allocator, compiled
with g++ from the library's own header and driven by random alloc/free
sequences (no GPU)."""
import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HDR = os.path.join(ROOT, "paper_1104_3830_amd", "csrc", "sk_alloc.h")

PROG = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include "HDR"
int main() {
    std::mt19937_64 rng(7);
    for (int trial = 0; trial < 50; ++trial) {
        sk::RangeAlloc a;
        const size_t base = 4096, cap = (size_t)1 << 24;
        a.init(base, cap);
        struct B { size_t off, len; };
        std::vector<B> live;
        for (int step = 0; step < 2000; ++step) {
            if (live.empty() || rng() % 3) {
                size_t len = 1 + rng() % (1 << 18);
                size_t off;
                if (a.alloc(len, off)) {
                    if (off < base || off + len > cap || off % 256) { printf("bounds\n"); return 1; }
                    for (auto &b : live)
                        if (off < b.off + b.len && b.off < off + len) { printf("overlap\n"); return 1; }
                    live.push_back({off, len});
                }
            } else {
                size_t k = rng() % live.size();
                a.release(live[k].off, live[k].len);
                live.erase(live.begin() + k);
            }
        }
        for (auto &b : live) a.release(b.off, b.len);
        if (a.free_.size() != 1 || a.free_bytes() != cap - base) { printf("coalesce\n"); return 1; }
    }
    printf("ok\n");
    return 0;
}
"""


def test_range_alloc_no_overlap_and_full_coalescing(tmp_path):
    src = tmp_path / "t.cpp"
    src.write_text(PROG.replace("HDR", HDR))
    exe = tmp_path / "t"
    subprocess.run(["g++", "-O2", "-std=c++17", str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True)
    assert out.returncode == 0 and out.stdout.strip() == "ok", out.stdout
