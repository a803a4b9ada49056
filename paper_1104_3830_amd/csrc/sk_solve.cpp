// The whole path for one instance, with the adaptive loop of Algorithm
// alg:alg1 (Section 4.2): continuation in p; at the end of each stage the FP64
// certificate (Proposition prop:aoc), the reduced matrix B (eq. matrixred),
// an exact optimal assignment of B on the host and the ratio gamma
// (eq. optratio); it stops at the first stage whose gamma is within the
// required ratio.
//
// When every stage is evaluated, the device stage controller pauses at each
// stage end (Inst::pause); the host evaluates the stage and either stops or
// moves to the next p with p^-1 log u and p^-1 log v held fixed.
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "sk_runtime.h"

namespace sk {
namespace {

struct StageResult {
    bool feasible = false;
    int p = 0;
    double t = 0;
    double log_gamma = INFINITY;
    int64_t weight = 0;
    int64_t nnz = 0;
    std::vector<int32_t> perm;
    sk_report rep{};
};

// B at threshold t from the committed potentials of instance 0, its CSR on
// the host, and an exact optimum of B (feasible = B has a perfect matching).
// With counted, the row lengths of B are already in B.d_counts, their scan in
// d_rp and the entry count in ctx->h_nnz[0] (the FP64 check made them).
// d_hint: per row the column of its largest x_ij, the start of the matching.
sk_status reduce_and_solve(sk_ctx *ctx, Batch &B, Bump &rest, int64_t *d_rp, const int32_t *d_hint,
                           double t, bool counted, StageResult &r) {
    const Inst &I = B.h_insts[0];
    const int n = I.n;
    const double logt = std::log(t);
    const int nunits = (int)B.h_rows.size();
    const size_t lds = gq_lds_bytes(n);
    // n > kLdsMaxN: the CSR passes read (G_j, gam_j) packed in I.colpack
    const int gcol = I.colpack != nullptr;
    if (gcol) HIPCHK(ctx, launch_col_pack(B.d_insts, 0, n, 1, ctx->stream));
    if (!counted) {
        HIPCHK(ctx, PROF(ctx, KID_PRUNE_COUNT, launch_prune_count(B.d_insts, B.d_rows, nunits, B.row_grid,
                                                                 logt, B.d_counts, lds, I.nt, gcol,
                                                                 ctx->stream)));
        HIPCHK(ctx, PROF(ctx, KID_SCAN, launch_scan(B.d_counts, d_rp, n, ctx->stream, B.d_nnz)));
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_nnz, B.d_nnz, sizeof(int64_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    }
    const int64_t nnz = ctx->h_nnz[0];
    // the host copy goes to pinned memory kept by the context: one DMA per
    // array, and no fresh pages to fault in on every call
    const size_t o_hint = align_up(sizeof(int64_t) * ((size_t)n + 1), 256);
    const size_t o_col = o_hint + align_up(sizeof(int32_t) * (size_t)n, 256);
    const size_t o_w = o_col + align_up(sizeof(int32_t) * (size_t)nnz, 256);
    const size_t need = o_w + align_up(sizeof(int16_t) * (size_t)nnz, 256);
    if (need > ctx->h_csr_bytes) {
        if (ctx->h_csr) HIPCHK(ctx, hipHostFree(ctx->h_csr));
        ctx->h_csr = nullptr;
        ctx->h_csr_bytes = 0;
        const size_t bytes = std::max(need, need / 2 * 3);  // room to grow
        HIPCHK(ctx, hipHostMalloc((void **)&ctx->h_csr, bytes, hipHostMallocDefault));
        ctx->h_csr_bytes = bytes;
    }
    int64_t *rp = reinterpret_cast<int64_t *>(ctx->h_csr);
    int32_t *hint = reinterpret_cast<int32_t *>(ctx->h_csr + o_hint);
    int32_t *col = reinterpret_cast<int32_t *>(ctx->h_csr + o_col);
    int16_t *w = reinterpret_cast<int16_t *>(ctx->h_csr + o_w);
    if (nnz > 0) {
        Bump tmp = rest;  // the entries are scratch until copied out
        int32_t *d_col = tmp.take<int32_t>((size_t)nnz);
        int16_t *d_w = tmp.take<int16_t>((size_t)nnz);
        if (!d_col || !d_w)
            return fail(ctx, SK_ENOMEM, "the reduced matrix keeps %lld entries; the arena cannot hold them",
                        (long long)nnz);
        HIPCHK(ctx, PROF(ctx, KID_PRUNE_FILL, launch_prune_fill(B.d_insts, B.d_rows, nunits, B.row_grid,
                                                               logt, d_rp, d_col, d_w, lds, I.nt, gcol,
                                                               ctx->stream)));
        HIPCHK(ctx, hipMemcpyAsync(col, d_col, sizeof(int32_t) * (size_t)nnz,
                                   hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(w, d_w, sizeof(int16_t) * (size_t)nnz, hipMemcpyDeviceToHost,
                                   ctx->stream));
    }
    HIPCHK(ctx, hipMemcpyAsync(rp, d_rp, sizeof(int64_t) * ((size_t)n + 1),
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(hint, d_hint, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    sk_csr csr{n, nnz, rp, col, w};
    r.perm.assign((size_t)n, -1);
    r.t = t;
    r.nnz = nnz;
    const sk_status s = solve_reduced_seeded(&csr, hint, r.perm.data(), &r.weight);
    if (s == SK_EINFEASIBLE) {
        r.feasible = false;
        return SK_OK;
    }
    if (s != SK_OK) return fail(ctx, s, "exact solve of the reduced matrix rejected its CSR");
    r.feasible = true;
    return SK_OK;
}

}  // namespace
}  // namespace sk

using namespace sk;

size_t sk_solve_arena_bytes(int32_t n, int32_t storage, int64_t max_kept) {
    if (n < 1 || n > kMaxN || max_kept < 0) return 0;
    return sk_arena_bytes(n, storage) + align_up(sizeof(int64_t) * ((size_t)n + 1), 256) +
           align_up(sizeof(int32_t) * (size_t)n, 256) +
           align_up(sizeof(int32_t) * (size_t)max_kept, 256) +
           align_up(sizeof(int16_t) * (size_t)max_kept, 256) + 1024;
}

extern "C" sk_status sk_solve(sk_ctx *ctx, const int16_t *W, int32_t n, const sk_params *params,
                              void *potentials, int32_t *perm, int64_t *weight, sk_report *report) {
    if (!ctx) return SK_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> g(ctx->mu);
    if (serving(ctx)) return fail(ctx, SK_EINVAL, "context is serving; blocking calls are disabled");
    ctx->absorbs = 0;
    sk_status st = check_params(ctx, params);
    if (st != SK_OK) return st;
    if (!W || !potentials || !perm || !weight) return fail(ctx, SK_EINVAL, "null argument");
    if ((st = check_size(ctx, n, params)) != SK_OK) return st;
    if (!(params->threshold > 0.0)) return fail(ctx, SK_EINVAL, "threshold must be > 0");
    if (params->fused && params->storage == SK_W_I16 && (n % 8 != 0 || (uintptr_t)W % 16 != 0))
        return fail(ctx, SK_EINVAL, "the single-pass iteration over int16 W needs n %% 8 == 0");
    if ((st = check_range(ctx, params)) != SK_OK) return st;
    HIPCHK(ctx, hipSetDevice(ctx->device));
    Bump bump{ctx->arena, ctx->arena_bytes};
    Batch &B = ctx->scratch_batch;
    int64_t pitch = n;
    const int16_t *Ws[1] = {W};
    // gamma <= opt_ratio is the stopping rule (reading of Algorithm alg:alg1);
    // opt_ratio < 1 asks for one evaluation, at the last p, and the log-domain
    // device controller then runs the whole ladder without pausing
    const bool adaptive = params->opt_ratio >= 1.0;
    const double log_ratio = adaptive ? std::log(params->opt_ratio) : 0.0;
    const bool kpath = params->storage != SK_W_I16;
    if ((st = plan_batch(ctx, bump, 1, Ws, &pitch, &n, params, B)) != SK_OK) return st;
    B.h_insts[0].pause = (adaptive && !kpath && params->method == SK_SINKHORN) ? 1 : 0;
    if ((st = upload_batch(ctx, B)) != SK_OK) return st;
    void *pots[1] = {potentials};
    if ((st = start_batch(ctx, B, params, pots)) != SK_OK) return st;
    StageResult best;
    bool have_best = false, reached = false;
    int evaluated = 0;

    // the end of one stage: certificate, B, exact optimum of B, gamma
    auto evaluate = [&](const Ctl &c, bool last, bool &stop) -> sk_status {
        stop = false;
        if (!(adaptive || last)) return SK_OK;
        StageResult r;
        r.p = c.p;
        fill_report(c, &r.rep);
        Bump rest = bump;
        int64_t *d_rp = rest.take<int64_t>((size_t)n + 1);
        int32_t *d_hint = rest.take<int32_t>((size_t)n);
        if (!d_rp || !d_hint)
            return fail(ctx, SK_ENOMEM, "arena too small for the reduced matrix (row pointers)");
        // FP64 certificate, row lengths of B at t and their scan: one sync
        double t = params->threshold;
        const CheckCounts cc{std::log(t), B.d_counts, d_hint};
        sk_status s2 = enqueue_check(ctx, B, 0, &cc);
        if (s2 != SK_OK) return s2;
        HIPCHK(ctx, PROF(ctx, KID_SCAN, launch_scan(B.d_counts, d_rp, n, ctx->stream, B.d_nnz)));
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_checkout, B.d_checkout, 4 * sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_nnz, B.d_nnz, sizeof(int64_t), hipMemcpyDeviceToHost,
                                   ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        report_from_check(ctx->h_checkout, c.p, &r.rep);
        // a B with no perfect matching at the last p: lower t tenfold, at most three times
        for (int tries = 0;; ++tries) {
            if ((s2 = reduce_and_solve(ctx, B, rest, d_rp, d_hint, t, tries == 0, r)) != SK_OK)
                return s2;
            if (r.feasible || !last || tries == 3) break;
            t /= 10.0;
        }
        ++evaluated;
        if (r.feasible) {
            r.log_gamma = r.rep.ub - (double)r.weight;
            if (!have_best || r.log_gamma < best.log_gamma) {
                if ((s2 = copy_potentials_out(ctx, B, 0, potentials)) != SK_OK) return s2;
                best = std::move(r);
                have_best = true;
            }
            if (!adaptive || best.log_gamma <= log_ratio) {
                reached = true;
                stop = true;
            }
        }
        return SK_OK;
    };

    if (params->method == SK_NEWTON) {
        // Newton scaling ends every stage on the host anyway
        const StageHook hook = [&](bool &stop) {
            const Ctl &c = ctx->h_ctl[0];
            return evaluate(c, c.stage + 1 >= params->n_p, stop);
        };
        if ((st = run_newton_i16(ctx, B, params, bump, &hook)) != SK_OK) return st;
        if ((st = read_ctl(ctx, B)) != SK_OK) return st;
    } else if (kpath) {
        // stored K: the controller pauses at every stage end anyway
        const StageHook hook = [&](bool &stop) {
            const Ctl &c = ctx->h_ctl[0];
            return evaluate(c, c.stage + 1 >= params->n_p, stop);
        };
        if ((st = run_single_k(ctx, B, params, &hook)) != SK_OK) return st;
        if ((st = read_ctl(ctx, B)) != SK_OK) return st;
    } else {
        int stage = 0;
        for (;;) {
            if ((st = run_batch_i16(ctx, B, params, stage)) != SK_OK) return st;
            const Ctl c = ctx->h_ctl[0];
            if (c.state == ST_ERROR) break;
            if (c.state != ST_STAGE_END && c.state != ST_DONE)
                return fail(ctx, SK_EDEVICE, "stage controller ended in state %d", c.state);
            stage = c.stage;
            const bool last = c.state == ST_DONE || stage + 1 >= params->n_p;
            bool stop = false;
            if ((st = evaluate(c, last, stop)) != SK_OK) return st;
            if (stop || last) break;
            HIPCHK(ctx, launch_advance(B.d_insts, 1, ctx->stream));
            stage += 1;
        }
    }
    const Ctl c = ctx->h_ctl[0];
    if (c.state == ST_ERROR || (c.err & (ERR_EMPTY_ROW | ERR_EMPTY_COL))) {
        if (report) {
            memset(report, 0, sizeof *report);
            fill_report(c, report);
            report->log_gamma = NAN;
            report->threshold_used = NAN;
        }
        if (c.err & ERR_NEWTON) return fail(ctx, SK_EDEVICE, "Newton scaling broke down");
        return fail(ctx, status_of(c), "a row or column of A has no entry");
    }
    if (!have_best) {
        if ((st = copy_potentials_out(ctx, B, 0, potentials)) != SK_OK) return st;
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    sk_report rep;
    memset(&rep, 0, sizeof rep);
    fill_report(c, &rep);  // work done over all stages run
    rep.absorbs = ctx->absorbs;
    if (have_best) {
        rep.residual_fp64 = best.rep.residual_fp64;
        rep.col_residual_fp64 = best.rep.col_residual_fp64;
        rep.residual_exact_fp64 = best.rep.residual_exact_fp64;
        rep.col_residual_exact_fp64 = best.rep.col_residual_exact_fp64;
        if (kpath && best.p == params->p_ladder[params->n_p - 1] && !std::isnan(ctx->k_res_rows)) {
            // the matrix the stored-K sweeps balance, K a b (before folding)
            rep.residual_fp64 = ctx->k_res_rows;
            rep.col_residual_fp64 = ctx->k_res_cols;
        }
        rep.ub = best.rep.ub;
        rep.residual_fp32 = best.rep.residual_fp32;
        rep.p_final = best.p;
        rep.nnz_kept = best.nnz;
        rep.log_gamma = best.log_gamma;
        rep.threshold_used = best.t;
        // integer weights: every permutation of A weighs at most ub, so
        // ub - w(B) < 1 leaves no room for a better one
        rep.optimal_proved = best.log_gamma < 1.0 - 1e-9 ? 1 : 0;
        memcpy(perm, best.perm.data(), sizeof(int32_t) * (size_t)n);
        *weight = best.weight;
    } else {
        rep.log_gamma = NAN;
        rep.threshold_used = NAN;
    }
    rep.stages_evaluated = evaluated;
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (report) *report = rep;
    if (!have_best)
        return fail(ctx, SK_EINFEASIBLE, "no reduced matrix had a perfect matching (last t = %g)",
                    params->threshold * 1e-3);
    if (!reached)
        return fail(ctx, SK_ENOCONV, "gamma = exp(%g) above opt_ratio %g after the last p",
                    best.log_gamma, params->opt_ratio);
    return SK_OK;
}
