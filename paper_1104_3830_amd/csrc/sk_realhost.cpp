// Host side of the real-valued log-weight path: sk_scale_real and
// sk_solve_real (Algorithm alg:alg1 with the prescaling of Section 4.1.1 and a
// real p).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <queue>
#include <vector>

#include "sk_hostsolve.h"
#include "sk_runtime.h"

namespace sk {
namespace {

constexpr int kMinmaxGrid = 256;

size_t real_shared_extra(int32_t n, int64_t max_kept) {
    return align_up(sizeof(float) * 3 * kMinmaxGrid, 256) +
           align_up(sizeof(int64_t) * ((size_t)n + 1), 256) + align_up(sizeof(int32_t) * (size_t)n, 256) +
           align_up(sizeof(int32_t) * (size_t)max_kept, 256) + align_up(sizeof(float) * (size_t)max_kept, 256) +
           1024;
}

// Argument checks, the range scan (NaN / +inf rejected, the prescaling
// factor and the common shift wref) and the plan of the one instance.
sk_status plan_real(sk_ctx *ctx, Bump &bump, const float *W, int32_t n, const sk_params *params, Batch &B) {
    sk_status st = check_params(ctx, params, true);
    if (st != SK_OK) return st;
    if (!W) return fail(ctx, SK_EINVAL, "null W");
    if (n < 1 || n > kLdsMaxN) return fail(ctx, SK_EINVAL, "n = %d outside [1, %d]", n, kLdsMaxN);
    HIPCHK(ctx, hipSetDevice(ctx->device));
    // range scan into scratch at the start of the arena (reused by the plan)
    Bump tmp = bump;
    float *d_part = tmp.take<float>(3 * (size_t)kMinmaxGrid);
    if (!d_part) return fail(ctx, SK_ENOMEM, "arena too small for the range scan");
    const int grid = std::min(kMinmaxGrid, n);
    HIPCHK(ctx, launch_real_minmax(W, n, n, grid, d_part, ctx->stream));
    float *h = reinterpret_cast<float *>(ctx->h_checkout);  // pinned, >= 3 * kMinmaxGrid floats
    HIPCHK(ctx, hipMemcpyAsync(h, d_part, sizeof(float) * 3 * (size_t)grid, hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    float lo = INFINITY, hi = -INFINITY;
    bool bad = false;
    for (int b = 0; b < grid; ++b) {
        lo = std::min(lo, h[3 * b]);
        hi = std::max(hi, h[3 * b + 1]);
        bad |= h[3 * b + 2] != 0.f;
    }
    if (bad) return fail(ctx, SK_EINVAL, "W holds a NaN or +inf (log-weights are finite or -inf)");
    if (!(hi >= lo)) return fail(ctx, SK_ENOSUPPORT, "W has no finite entry");
    const double range = (double)hi - (double)lo;
    const double pscale = params->prescale && range > 1.0 ? 1.0 / range : 1.0;
    // the potentials stay within a few p times the weight range: keep them
    // (and p w in the column rescue) well inside int32
    int pmax = 0;
    for (int s = 0; s < params->n_p; ++s) pmax = std::max(pmax, params->p_ladder[s]);
    if ((double)pmax * pscale * std::max(range, 1.0) > 1.0e8)
        return fail(ctx, SK_EINVAL, "p * (w_max - w_min) = %g exceeds 1e8", (double)pmax * pscale * range);
    const int64_t pitch = n;
    const int16_t *Ws[1] = {nullptr};
    B.h_insts.assign(1, Inst{});
    if (!carve_instance(bump, Ws[0], pitch, n, params, B.h_insts[0], W))
        return fail(ctx, SK_ENOMEM, "arena too small for the instance (n=%d)", n);
    B.h_insts[0].wref = hi;
    B.h_insts[0].pscale = pscale;
    return finish_tables(ctx, bump, B);
}

}  // namespace
}  // namespace sk

using namespace sk;

size_t sk_real_arena_bytes(int32_t n, int64_t max_kept) {
    if (n < 1 || n > kLdsMaxN || max_kept < 0) return 0;
    return instance_bytes(n, 1, SK_W_I16) + shared_bytes(1, &n) + real_shared_extra(n, max_kept) + 4096;
}

sk_status sk_scale_real(sk_ctx *ctx, const float *W, int32_t n, const sk_params *params,
                        void *potentials, sk_report *report) {
    if (!ctx) return SK_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> g(ctx->mu);
    if (serving(ctx)) return fail(ctx, SK_EINVAL, "context is serving; blocking calls are disabled");
    if (!params) return fail(ctx, SK_EINVAL, "params is NULL");
    if (!potentials) return fail(ctx, SK_EINVAL, "null potentials");
    ctx->absorbs = 0;
    Bump bump{ctx->arena, ctx->arena_bytes};
    Batch &B = ctx->scratch_batch;
    sk_status st = plan_real(ctx, bump, W, n, params, B);
    if (st != SK_OK) return st;
    if ((st = upload_batch(ctx, B)) != SK_OK) return st;
    void *pots[1] = {potentials};
    if ((st = start_batch(ctx, B, params, pots)) != SK_OK) return st;
    if ((st = run_batch_i16(ctx, B, params)) != SK_OK) return st;
    const Ctl c = ctx->h_ctl[0];
    sk_report rep;
    memset(&rep, 0, sizeof rep);
    fill_report(c, &rep);
    rep.p_scale = B.h_insts[0].pscale;
    rep.log_gamma = NAN;
    rep.threshold_used = NAN;
    const bool empty = (c.err & (ERR_EMPTY_ROW | ERR_EMPTY_COL)) != 0;
    if (!empty) {
        if ((st = enqueue_check(ctx, B, 0)) != SK_OK) return st;
        HIPCHK(ctx, hipMemcpyAsync(ctx->h_checkout, B.d_checkout, 4 * sizeof(double),
                                   hipMemcpyDeviceToHost, ctx->stream));
        HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
        // the deformed iteration's last p is unrounded on real-valued weights
        const double pl = params->deform_a > 0.0 ? c.preal : (double)c.p;
        report_from_check(ctx->h_checkout, pl * rep.p_scale, &rep, n, B.h_insts[0].wref);
    }
    if ((st = copy_potentials_out(ctx, B, 0, potentials)) != SK_OK) return st;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (report) *report = rep;
    const sk_status s = status_of(c);
    if (s == SK_ENOSUPPORT) return fail(ctx, s, "a row or column of A has no entry");
    if (s == SK_ENOCONV) return fail(ctx, s, "a stage hit max_iters_per_stage");
    return s;
}

sk_status sk_solve_real(sk_ctx *ctx, const float *W, int32_t n, const sk_params *params,
                        void *potentials, int32_t *perm, double *weight, sk_report *report) {
    if (!ctx) return SK_EINVAL;
    const auto t0 = std::chrono::steady_clock::now();
    std::lock_guard<std::mutex> g(ctx->mu);
    if (serving(ctx)) return fail(ctx, SK_EINVAL, "context is serving; blocking calls are disabled");
    if (!params) return fail(ctx, SK_EINVAL, "params is NULL");
    if (!potentials || !perm || !weight) return fail(ctx, SK_EINVAL, "null argument");
    if (!(params->threshold > 0.0)) return fail(ctx, SK_EINVAL, "threshold must be > 0");
    ctx->absorbs = 0;
    Bump bump{ctx->arena, ctx->arena_bytes};
    Batch &B = ctx->scratch_batch;
    sk_status st = plan_real(ctx, bump, W, n, params, B);
    if (st != SK_OK) return st;
    const bool adaptive = params->opt_ratio >= 1.0;
    const double log_ratio = adaptive ? std::log(params->opt_ratio) : 0.0;
    B.h_insts[0].pause = adaptive ? 1 : 0;
    const double pscale = B.h_insts[0].pscale, wref = B.h_insts[0].wref;
    const double gscale = params->prescale ? pscale : 1.0;  // gamma of the prescaled matrix
    if ((st = upload_batch(ctx, B)) != SK_OK) return st;
    void *pots[1] = {potentials};
    if ((st = start_batch(ctx, B, params, pots)) != SK_OK) return st;

    struct Best {
        bool have = false;
        int p = 0;
        double t = 0, log_gamma = INFINITY, weight = 0;
        int64_t nnz = 0;
        std::vector<int32_t> perm;
        sk_report rep{};
    } best;
    bool reached = false;
    int evaluated = 0;
    auto evaluate = [&](const Ctl &c, bool last, bool &stop) -> sk_status {
        stop = false;
        if (!(adaptive || last)) return SK_OK;
        sk_report rep;
        memset(&rep, 0, sizeof rep);
        fill_report(c, &rep);
        Bump rest = bump;
        int64_t *d_rp = rest.take<int64_t>((size_t)n + 1);
        int32_t *d_hint = rest.take<int32_t>((size_t)n);
        if (!d_rp || !d_hint) return fail(ctx, SK_ENOMEM, "arena too small for the reduced matrix");
        double t = params->threshold;
        std::vector<int64_t> rp((size_t)n + 1);
        std::vector<int32_t> hint((size_t)n), colh;
        std::vector<float> wh;
        std::vector<int32_t> pm((size_t)n);
        double wB = 0.0;
        bool feasible = false;
        int64_t nnz = 0;
        // a B with no perfect matching at the last p: lower t tenfold, at most three times
        for (int tries = 0;; ++tries) {
            const CheckCounts cc{std::log(t), B.d_counts, d_hint};
            sk_status s2 = enqueue_check(ctx, B, 0, &cc);
            if (s2 != SK_OK) return s2;
            HIPCHK(ctx, PROF(ctx, KID_SCAN, launch_scan(B.d_counts, d_rp, n, ctx->stream, B.d_nnz)));
            HIPCHK(ctx, hipMemcpyAsync(ctx->h_checkout, B.d_checkout, 4 * sizeof(double),
                                       hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(ctx->h_nnz, B.d_nnz, sizeof(int64_t), hipMemcpyDeviceToHost,
                                       ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            report_from_check(ctx->h_checkout, (params->deform_a > 0.0 ? c.preal : (double)c.p) * pscale, &rep,
                              n, wref);
            nnz = ctx->h_nnz[0];
            Bump tmp = rest;
            int32_t *d_col = tmp.take<int32_t>((size_t)std::max<int64_t>(nnz, 1));
            float *d_w = tmp.take<float>((size_t)std::max<int64_t>(nnz, 1));
            if (!d_col || !d_w)
                return fail(ctx, SK_ENOMEM, "the reduced matrix keeps %lld entries; the arena cannot hold them",
                            (long long)nnz);
            colh.resize((size_t)nnz);
            wh.resize((size_t)nnz);
            if (nnz > 0) {
                HIPCHK(ctx, PROF(ctx, KID_PRUNE_FILL,
                                 launch_prune_fill_real(B.d_insts, B.d_rows, (int)B.h_rows.size(), B.row_grid,
                                                        std::log(t), d_rp, d_col, d_w, n, ctx->stream)));
                HIPCHK(ctx, hipMemcpyAsync(colh.data(), d_col, sizeof(int32_t) * (size_t)nnz,
                                           hipMemcpyDeviceToHost, ctx->stream));
                HIPCHK(ctx, hipMemcpyAsync(wh.data(), d_w, sizeof(float) * (size_t)nnz, hipMemcpyDeviceToHost,
                                           ctx->stream));
            }
            HIPCHK(ctx, hipMemcpyAsync(rp.data(), d_rp, sizeof(int64_t) * ((size_t)n + 1),
                                       hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(ctx, hipMemcpyAsync(hint.data(), d_hint, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToHost,
                                       ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            s2 = solve_real_impl(n, rp.data(), colh.data(), wh.data(), hint.data(), pm.data(), &wB);
            if (s2 == SK_OK) {
                feasible = true;
                break;
            }
            if (s2 != SK_EINFEASIBLE) return fail(ctx, s2, "exact solve of the reduced matrix rejected its CSR");
            if (!last || tries == 3) break;
            t /= 10.0;
        }
        ++evaluated;
        if (feasible) {
            const double lg = gscale * (rep.ub - wB);
            if (!best.have || lg < best.log_gamma) {
                sk_status s2 = copy_potentials_out(ctx, B, 0, potentials);
                if (s2 != SK_OK) return s2;
                best.have = true;
                best.p = c.p;
                best.t = t;
                best.log_gamma = lg;
                best.weight = wB;
                best.nnz = nnz;
                best.perm = pm;
                best.rep = rep;
            }
            if (!adaptive || best.log_gamma <= log_ratio) {
                reached = true;
                stop = true;
            }
        }
        return SK_OK;
    };

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
    const Ctl c = ctx->h_ctl[0];
    if (c.state == ST_ERROR || (c.err & (ERR_EMPTY_ROW | ERR_EMPTY_COL))) {
        if (report) {
            memset(report, 0, sizeof *report);
            fill_report(c, report);
            report->log_gamma = NAN;
            report->threshold_used = NAN;
            report->p_scale = pscale;
        }
        return fail(ctx, status_of(c), "a row or column of A has no entry");
    }
    if (!best.have) {
        if ((st = copy_potentials_out(ctx, B, 0, potentials)) != SK_OK) return st;
    }
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    sk_report rep;
    memset(&rep, 0, sizeof rep);
    fill_report(c, &rep);  // work done over all stages run
    rep.p_scale = pscale;
    if (best.have) {
        rep.residual_fp64 = best.rep.residual_fp64;
        rep.col_residual_fp64 = best.rep.col_residual_fp64;
        rep.residual_exact_fp64 = best.rep.residual_exact_fp64;
        rep.col_residual_exact_fp64 = best.rep.col_residual_exact_fp64;
        rep.ub = best.rep.ub;
        rep.residual_fp32 = best.rep.residual_fp32;
        rep.p_final = best.p;
        rep.nnz_kept = best.nnz;
        rep.log_gamma = best.log_gamma;
        rep.threshold_used = best.t;
        memcpy(perm, best.perm.data(), sizeof(int32_t) * (size_t)n);
        *weight = best.weight;
    } else {
        rep.log_gamma = NAN;
        rep.threshold_used = NAN;
    }
    rep.stages_evaluated = evaluated;
    rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    if (report) *report = rep;
    if (!best.have)
        return fail(ctx, SK_EINFEASIBLE, "no reduced matrix had a perfect matching");
    if (!reached)
        return fail(ctx, SK_ENOCONV, "gamma = exp(%g) above opt_ratio %g after the last p", best.log_gamma,
                    params->opt_ratio);
    return SK_OK;
}
