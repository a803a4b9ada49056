// Newton scaling of one instance (Section 5.2, the Knight-Ruiz method cited
// there), stage by stage over the p ladder. Each stage solves
// x o (S x) = 1 for the symmetric embedding S = [[0, X], [X^T, 0]] of the
// matrix X scaled by the stage's starting potentials, by Newton steps whose
// linear systems are solved by preconditioned conjugate gradients; the
// iteration runs on the device (product kernels + four short phase kernels
// per step, the state in a device control block) and the host only launches
// blocks of steps and reads the control block. The scalings found are folded into the
// potentials, then p moves on with p^-1 log u and p^-1 log v held fixed.
#include <vector>

#include "sk_runtime.h"

namespace sk {

sk_status run_newton_i16(sk_ctx *ctx, Batch &B, const sk_params *prm, Bump &bump,
                         const StageHook *hook) {
    const Inst &I = B.h_insts[0];
    const int n = I.n;
    const size_t n2 = 2 * (size_t)n;
    NtCtl *d_nt = bump.take<NtCtl>(2);  // double-buffered by phase parity; [1] is current
    NtVec V{};
    float **vecs[] = {&V.q, &V.sd, &V.x, &V.v, &V.r, &V.z, &V.d, &V.y, &V.w};
    for (float **p : vecs) *p = bump.take<float>(n2);
    for (float **p : vecs)
        if (!*p) return fail(ctx, SK_ENOMEM, "arena too small for the Newton vectors");
    V.parts = bump.take<double>((size_t)(kNtPhases + 1) * kNtMaxGroups * 4);
    if (!d_nt || !V.parts) return fail(ctx, SK_ENOMEM, "arena too small for the Newton state");
    const std::vector<float> ones(n2, 1.f);
    const int check = std::max(1, prm->check_every);
    const int64_t bound = prm->max_iters_per_stage / check + 16;
    for (int s = 0; s < prm->n_p; ++s) {
        sk_status st = read_ctl(ctx, B);
        if (st != SK_OK) return st;
        if (ctx->h_ctl[0].state == ST_ERROR || (ctx->h_ctl[0].err & (ERR_EMPTY_ROW | ERR_EMPTY_COL)))
            return SK_OK;
        NtCtl init{};
        init.mode = NT_OUTER;
        init.done = NT_RUN;
        init.first = 1;
        init.max_products = prm->max_iters_per_stage;
        init.tol = prm->tol;
        init.lo = 0.1;
        init.hi = 3.0;
        init.eta_max = 0.1;
        init.g = 0.9;
        init.eta = 0.1;
        const NtCtl init2[2] = {init, init};
        HIPCHK(ctx, hipMemcpyAsync(d_nt, init2, sizeof init2, hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(V.x, ones.data(), sizeof(float) * n2, hipMemcpyHostToDevice,
                                   ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(V.q, ones.data(), sizeof(float) * n2, hipMemcpyHostToDevice,
                                   ctx->stream));
        const size_t pstart = ctx->prof.pending.size();
        NtCtl h{};
        for (int64_t rounds = 0;; ++rounds) {
            for (int k = 0; k < check; ++k) {
                HIPCHK(ctx, PROF(ctx, KID_NT_PRODUCT,
                                 launch_nt_product(B.d_insts, B.d_rows, (int)B.h_rows.size(),
                                                   B.row_grid, B.row_lds, B.d_cols,
                                                   (int)B.h_cols.size(), B.col_grid, d_nt, V, n,
                                                   B.h_insts[0].nt, ctx->stream)));
                HIPCHK(ctx, PROF(ctx, KID_NT_STEP, launch_nt_step(B.d_insts, d_nt, V, n, ctx->stream)));
            }
            HIPCHK(ctx, hipMemcpyAsync(&h, d_nt + 1, sizeof h, hipMemcpyDeviceToHost, ctx->stream));
            HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
            if (h.done != NT_RUN) break;
            if (rounds > bound) return fail(ctx, SK_EDEVICE, "Newton controller did not terminate");
        }
        if (ctx->prof.on) {
            // launches after the iteration ended returned at once
            const int64_t work = h.products;
            ctx->prof.retag(pstart, KID_NT_PRODUCT,
                            [=](int64_t t) { return t >= work ? (int)KID_NT_PRODUCT_IDLE : -1; });
            ctx->prof.retag(pstart, KID_NT_STEP,
                            [=](int64_t t) { return t >= work ? (int)KID_NT_STEP_IDLE : -1; });
        }
        const bool last = s + 1 >= prm->n_p;
        HIPCHK(ctx, launch_nt_fold(B.d_insts, d_nt, V, n, last ? 1 : 0, ctx->stream));
        if ((st = read_ctl(ctx, B)) != SK_OK) return st;
        if (ctx->h_ctl[0].state == ST_ERROR) return SK_OK;
        if (hook) {
            bool stop = false;
            if ((st = (*hook)(stop)) != SK_OK) return st;
            if (stop) return SK_OK;
        }
        if (!last) HIPCHK(ctx, launch_advance(B.d_insts, 1, ctx->stream));
    }
    return SK_OK;
}

}  // namespace sk
