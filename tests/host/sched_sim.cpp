// The served path's admission policy (sk_sched.h) driven by a mock executor:
// requests of random footprints arrive at random ticks; copies into device
// regions and the Sinkhorn work of admitted requests take random numbers of
// ticks; finished requests release their regions. The tick follows the
// serving loop: admission, copies started, completed copies taken in
// admission order, work, retirement. Checked at every tick: regions
// disjoint and inside the arena, the allocator's free bytes consistent with
// the live regions, the batch limit, FIFO admission, a device region taken
// at submission only when no earlier request waits for one, no region
// withheld from the queue's head while one would fit, and every refusal
// justified. After the arrivals stop, everything drains: every accepted
// request finishes exactly once and both allocators coalesce to one block.
// Built with AddressSanitizer and UndefinedBehaviorSanitizer by
// tests/test_host_sanitize.py; prints "ok" and exits 0 when every check holds.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <deque>
#include <memory>
#include <random>
#include <vector>

#include "sk_sched.h"

using sk::Entry;
using sk::RangeAlloc;

namespace {

int failures = 0;
#define CHECK(c)                                                        \
    do {                                                                \
        if (!(c)) {                                                     \
            std::printf("check failed at line %d: %s\n", __LINE__, #c); \
            ++failures;                                                 \
        }                                                               \
    } while (0)

struct Req {
    uint64_t id = 0;
    size_t len = 0, wbytes = 0;
    bool copying = false, loaded = false;
    int phase = 0;  // 0 queued, 1 in the batch, 3 done
    bool has_region = false;
    size_t off = 0;
    bool in_ring = false;
    size_t ring_off = 0;
    int copy_left = 0, work_left = 0;
    int finished = 0;
};

// alloc + release: would a block of len fit now (no lasting change)
bool fits(RangeAlloc &a, size_t len) {
    size_t off;
    if (!a.alloc(len, off)) return false;
    a.release(off, len);
    return true;
}

struct Sim {
    std::mt19937_64 rng;
    RangeAlloc dev, ring;
    bool with_ring;
    size_t base, cap, ring_cap, max_batch, max_queue;
    std::vector<std::unique_ptr<Req>> all;
    std::deque<Req *> queue, loading;
    std::vector<Req *> active;
    int staged_waiting = 0;
    uint64_t next_id = 1, last_admitted = 0;
    size_t refused = 0, placed_at_submit = 0;

    Sim(uint64_t seed, bool ring_on, size_t cap_, size_t ring_cap_, size_t batch, size_t queue_max)
        : rng(seed), with_ring(ring_on), base(4096), cap(cap_), ring_cap(ring_cap_), max_batch(batch),
          max_queue(queue_max) {
        dev.init(base, cap);
        ring.init(0, ring_cap);
    }

    int uni(int lo, int hi) { return std::uniform_int_distribution<int>(lo, hi)(rng); }

    void submit() {
        // footprints log-uniform over three decades, some near the arena size
        const double e = std::uniform_real_distribution<double>(10.0, 20.5)(rng);
        const size_t len = (size_t)std::exp2(e);
        if (len + base > cap) return;  // sk_submit refuses these before planning
        const size_t wbytes = len / 2 + 1;
        const size_t dev_free = dev.free_bytes(), ring_free = ring.free_bytes();
        const int waiting_before = staged_waiting;
        const size_t queued_before = queue.size();
        const bool ring_fit = with_ring && fits(ring, wbytes);
        const bool dev_fit = fits(dev, len);
        const sk::EntryPlan ep = sk::plan_entry(with_ring ? &ring : nullptr, dev, queue.size(), max_queue,
                                                staged_waiting, wbytes, len);
        if (ep.kind == Entry::Again) {
            ++refused;
            CHECK(dev.free_bytes() == dev_free && ring.free_bytes() == ring_free);
            CHECK(queued_before >= max_queue || (with_ring && !ring_fit && (waiting_before > 0 || !dev_fit)));
            return;
        }
        CHECK(queued_before < max_queue);
        auto r = std::make_unique<Req>();
        r->id = next_id++;
        r->len = len;
        r->wbytes = wbytes;
        const bool placed = ep.kind == Entry::RingAndDevice || ep.kind == Entry::DeviceOnly;
        if (placed) {
            CHECK(waiting_before == 0);
            r->has_region = true;
            r->off = ep.dev_off;
            ++placed_at_submit;
        } else {
            CHECK(waiting_before > 0 || !dev_fit);
        }
        if (ep.kind == Entry::RingAndDevice || ep.kind == Entry::RingOnly) {
            CHECK(with_ring);
            r->in_ring = true;
            r->ring_off = ep.ring_off;
        } else {
            CHECK(!ring_fit);
        }
        if (ep.kind == Entry::Heap) CHECK(!with_ring);
        switch (ep.kind) {
        case Entry::RingAndDevice:
            r->copying = true;
            r->copy_left = uni(0, 3);
            break;
        case Entry::DeviceOnly:
            r->loaded = true;  // a synchronous copy straight into the region
            break;
        default:
            ++staged_waiting;  // RingOnly, Heap: W waits on the host
        }
        queue.push_back(r.get());
        all.push_back(std::move(r));
    }

    void tick(bool arrivals) {
        if (arrivals) {
            const int k = uni(0, 4);
            for (int q = 0; q < k; ++q) submit();
        }
        // admission: the admitted requests are a prefix of the queue, and
        // each list keeps queue order
        std::vector<uint64_t> before;
        for (Req *r : queue) before.push_back(r->id);
        std::vector<Req *> fresh, to_copy;
        sk::admit_fifo(queue, active.size() + loading.size(), max_batch, dev, staged_waiting, fresh,
                       to_copy, [](Req *r, size_t off) {
                           r->has_region = true;
                           r->off = off;
                       });
        const size_t popped = before.size() - queue.size();
        CHECK(popped == fresh.size() + to_copy.size());
        std::vector<uint64_t> got;
        for (Req *r : to_copy) got.push_back(r->id);
        for (Req *r : fresh) got.push_back(r->id);
        CHECK(std::is_sorted(got.begin(), got.begin() + to_copy.size()));
        CHECK(std::is_sorted(got.begin() + to_copy.size(), got.end()));
        std::sort(got.begin(), got.end());
        CHECK(std::equal(got.begin(), got.end(), before.begin()));
        if (!got.empty()) {
            CHECK(got.front() > last_admitted);
            last_admitted = got.back();
        }
        // the head stays queued only for a full batch or a region that does not fit
        if (!queue.empty() && active.size() + loading.size() + fresh.size() + to_copy.size() < max_batch) {
            Req *h = queue.front();
            CHECK(!h->copying && !h->loaded && !h->has_region);
            CHECK(!fits(dev, h->len));
        }
        for (Req *r : to_copy) {
            if (!r->copying) {
                r->copying = true;
                r->copy_left = uni(0, 3);
            }
            loading.push_back(r);
        }
        // copies complete in any order; they are taken in admission order
        for (Req *r : loading)
            if (r->copy_left > 0) --r->copy_left;
        while (!loading.empty() && loading.front()->copy_left == 0) {
            Req *r = loading.front();
            loading.pop_front();
            if (r->in_ring) {
                ring.release(r->ring_off, r->wbytes);
                r->in_ring = false;
            }
            r->copying = false;
            r->loaded = true;
            fresh.push_back(r);
        }
        for (Req *r : fresh) {
            CHECK(r->has_region && r->loaded);
            r->work_left = uni(1, 6);
            active.push_back(r);
        }
        // work and retirement
        std::vector<Req *> keep;
        for (Req *r : active) {
            if (--r->work_left > 0) {
                keep.push_back(r);
                continue;
            }
            dev.release(r->off, r->len);
            r->has_region = false;
            r->phase = 3;
            ++r->finished;
        }
        active.swap(keep);
        check_state();
    }

    void check_state() {
        CHECK(active.size() + loading.size() <= max_batch);
        CHECK(queue.size() <= max_queue);
        // live regions: disjoint, inside the arena, and the allocator agrees
        std::vector<std::pair<size_t, size_t>> live;
        size_t live_ring = 0;
        for (auto &p : all) {
            if (p->has_region) live.push_back({p->off, RangeAlloc::round(p->len)});
            if (p->in_ring) live_ring += RangeAlloc::round(p->wbytes);
        }
        std::sort(live.begin(), live.end());
        size_t used = 0;
        for (size_t k = 0; k < live.size(); ++k) {
            CHECK(live[k].first >= base && live[k].first + live[k].second <= cap);
            CHECK(live[k].first % RangeAlloc::kGranule == 0);
            if (k + 1 < live.size()) CHECK(live[k].first + live[k].second <= live[k + 1].first);
            used += live[k].second;
        }
        CHECK(dev.free_bytes() + used == cap - base);
        CHECK(ring.free_bytes() + live_ring == ring_cap);
        int waiting = 0;
        for (Req *r : queue) waiting += (!r->copying && !r->loaded) ? 1 : 0;
        CHECK(waiting == staged_waiting);
    }

    void run(int arrival_ticks) {
        for (int t = 0; t < arrival_ticks; ++t) tick(true);
        int t = 0;
        while ((!queue.empty() || !loading.empty() || !active.empty()) && t < 100000) {
            tick(false);
            ++t;
        }
        CHECK(queue.empty() && loading.empty() && active.empty());
        CHECK(staged_waiting == 0);
        for (auto &p : all) CHECK(p->finished == 1 && p->phase == 3);
        CHECK(dev.free_.size() == 1 && dev.free_bytes() == cap - base);
        CHECK(ring.free_bytes() == ring_cap && ring.free_.size() <= 1);
    }
};

}  // namespace

int main() {
    size_t accepted = 0, refused = 0, placed = 0;
    for (int trial = 0; trial < 48; ++trial) {
        const bool with_ring = trial % 3 != 0;
        const size_t cap = (size_t)1 << (21 + trial % 4);       // 2 to 16 MiB of arena
        const size_t ring_cap = (size_t)1 << (20 + trial % 3);  // 1 to 4 MiB of ring
        const size_t batch = trial % 2 ? 512 : 6;
        const size_t qmax = trial % 4 == 1 ? 8 : 512;
        Sim s(1000 + trial, with_ring, cap, ring_cap, batch, qmax);
        s.run(300);
        accepted += s.all.size();
        refused += s.refused;
        placed += s.placed_at_submit;
    }
    // the runs exercised every branch: refusals, regions at submission and
    // regions handed out at admission
    CHECK(refused > 0 && placed > 0 && accepted > placed);
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ok accepted=%zu refused=%zu placed_at_submit=%zu\n", accepted, refused, placed);
    return 0;
}
