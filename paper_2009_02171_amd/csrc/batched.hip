// Batched restarted FGMRES (Sec. 3.3) over independent shells of different
// sizes: the shells advance in lock step, one Arnoldi step for all active
// shells at a time.  Each step is one replay of a captured hipGraph with one
// branch per active shell (preconditioner, operator, multi-dot, update and
// norm, copy of the dot products to the host), so the branches of small and
// large shells run concurrently and the host synchronises once per step for
// the whole batch.  The next basis vector is normalised on the device from the
// norm computed in the previous step, which keeps every node's arguments fixed
// for a given (active set, step index): graphs are captured once per pair and
// kept for later solves.
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <vector>

#include "common.h"
#include "krylov.h"
#include "profile.h"

namespace csd {

// v /= sqrt(nn2[0])  (nn2 > 0: a shell whose norm vanished has left the batch)
__global__ void k_scale_by_norm(double *__restrict__ v, int64_t n, const double *__restrict__ nn2) {
    const double sc = 1.0 / sqrt(nn2[0]);
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) v[i] *= sc;
}

struct BShell {
    const csdyn_opctx *ctx = nullptr;
    const csdyn_ras *pc = nullptr;
    int64_t n = 0;
    double *V = nullptr, *Z = nullptr, *r = nullptr, *tmp = nullptr, *partial = nullptr, *red = nullptr,
           *bproj = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t join = nullptr;
};

static void carve_shell(Carver &c, BShell &b, int m) {
    b.V = c.take<double>(size_t(m + 1) * b.n);
    b.Z = c.take<double>(size_t(m) * b.n);
    b.r = c.take<double>(b.n);
    b.tmp = c.take<double>(b.n);
    b.partial = c.take<double>(kPartialElems);
    b.red = c.take<double>(3 * kRedStride);
    b.bproj = c.take<double>(b.n);
}

}  // namespace csd

struct csdyn_batch {
    int nshell = 0, m = 30;
    csdyn_gmres_opts o{};
    std::vector<csd::BShell> sh;
    hipStream_t origin = nullptr;  // the steps are issued (and captured) here
    hipEvent_t fork = nullptr, ready = nullptr;
    double *hred = nullptr;  // pinned: [nshell][2 * kRedStride]
    std::map<std::pair<uint64_t, int>, hipGraphExec_t> graphs;
    ~csdyn_batch() {
        for (auto &kv : graphs) hipGraphExecDestroy(kv.second);
        for (auto &b : sh) {
            if (b.join) hipEventDestroy(b.join);
            if (b.st) hipStreamDestroy(b.st);
        }
        if (fork) hipEventDestroy(fork);
        if (ready) hipEventDestroy(ready);
        if (origin) hipStreamDestroy(origin);
        if (hred) hipHostFree(hred);
    }
};

namespace csd {

static int32_t check_batch(int32_t nshell, const csdyn_opctx *const *ops, const csdyn_ras *const *pcs,
                           const csdyn_gmres_opts *o) {
    if (nshell < 1 || nshell > 64 || !ops || !o) {
        set_error("batch: 1 <= nshell <= 64 and non-null shells and options required");
        return CSDYN_EINVAL;
    }
    if (o->restart < 1 || o->restart > kRedStride - 1 || o->maxit < 1) {
        set_error("batch: restart in [1, 32], maxit >= 1");
        return CSDYN_EINVAL;
    }
    if (o->orth != 0) { set_error("batch: classical Gram-Schmidt only (orth = 0)"); return CSDYN_EINVAL; }
    if (o->rhs_relative != 0 && o->rhs_relative != 1) { set_error("batch: rhs_relative must be 0 or 1"); return CSDYN_EINVAL; }
    for (int i = 0; i < nshell; ++i) {
        if (!ops[i]) { set_error("batch: null operator %d", i); return CSDYN_EINVAL; }
        if (pcs && pcs[i]) {
            if (ras_fine_ctx(pcs[i])->g.n != ops[i]->g.n || ras_fine_ctx(pcs[i])->g.nr != ops[i]->g.nr) {
                set_error("batch: preconditioner %d built for another grid", i);
                return CSDYN_EINVAL;
            }
            if (ras_levels(pcs[i]) != 1) {
                set_error("batch: shell %d: the two-level preconditioner synchronises with the host (inner solve); "
                          "batched solves take one-level preconditioners", i);
                return CSDYN_EINVAL;
            }
        }
    }
    return CSDYN_OK;
}

static size_t batch_bytes(int32_t nshell, const csdyn_opctx *const *ops, int m) {
    Carver c(nullptr);
    for (int i = 0; i < nshell; ++i) {
        BShell b;
        b.n = 24 * int64_t(ops[i]->g.n) * ops[i]->g.n * ops[i]->g.nr;
        carve_shell(c, b, m);
    }
    return c.off + 256;
}

// The launches of Arnoldi step j of one shell (also used eagerly).
static int32_t shell_step(csdyn_batch *bt, BShell &b, int j, hipStream_t s) {
    const int64_t n = b.n;
    double *vj = b.V + size_t(j) * n, *w = b.V + size_t(j + 1) * n, *zj = b.Z + size_t(j) * n;
    if (j > 0) {
        const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256));
        hipLaunchKernelGGL(k_scale_by_norm, dim3(unsigned(blocks)), dim3(256), 0, s, vj, n,
                           b.red + kRedStride + (kRedStride - 1));
        CSD_HIP(hipGetLastError());
    }
    if (b.pc) CSD_TRY(ras_apply_d(b.pc, vj, zj, s));
    else CSD_TRY(Vec<double>::copy(zj, vj, n, s));
    CSD_TRY(op_launch(b.ctx, zj, w, s));
    CSD_TRY(Vec<double>::mdot(b.V, n, j + 1, w, b.partial, b.red, s));
    CSD_TRY(Vec<double>::mupdate(w, b.V, n, j + 1, b.red, b.partial, b.red + kRedStride, s));
    const size_t i = size_t(&b - bt->sh.data());
    CSD_HIP(hipMemcpyAsync(bt->hred + i * 2 * kRedStride, b.red, sizeof(double) * 2 * kRedStride,
                           hipMemcpyDeviceToHost, s));
    return CSDYN_OK;
}

// Step j for the shells in `mask`, forked from s0 onto the shells' streams and joined back.
static int32_t issue_step(csdyn_batch *bt, uint64_t mask, int j, hipStream_t s0) {
    CSD_HIP(hipEventRecord(bt->fork, s0));
    for (int i = 0; i < bt->nshell; ++i) {
        if (!(mask >> i & 1)) continue;
        BShell &b = bt->sh[i];
        CSD_HIP(hipStreamWaitEvent(b.st, bt->fork, 0));
        CSD_TRY(shell_step(bt, b, j, b.st));
        CSD_HIP(hipEventRecord(b.join, b.st));
        CSD_HIP(hipStreamWaitEvent(s0, b.join, 0));
    }
    return CSDYN_OK;
}

static int32_t graph_for(csdyn_batch *bt, uint64_t mask, int j, hipStream_t s0, hipGraphExec_t &out) {
    auto key = std::make_pair(mask, j);
    auto it = bt->graphs.find(key);
    if (it != bt->graphs.end()) { out = it->second; return CSDYN_OK; }
    CSD_HIP(hipStreamBeginCapture(s0, hipStreamCaptureModeRelaxed));
    prof_suspend(true);
    const int32_t rc = issue_step(bt, mask, j, s0);
    prof_suspend(false);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(s0, &g);
    if (rc != CSDYN_OK) {
        if (g) hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) {
        set_error("batch: graph capture failed: %s", hipGetErrorString(e));
        return CSDYN_EHIP;
    }
    hipGraphExec_t ex = nullptr;
    const hipError_t ei = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (ei != hipSuccess) {
        set_error("batch: graph instantiation failed: %s", hipGetErrorString(ei));
        return CSDYN_EHIP;
    }
    bt->graphs[key] = ex;
    out = ex;
    return CSDYN_OK;
}

static int32_t dev_norm(BShell &b, const double *v, double &out, hipStream_t s) {
    CSD_TRY(Vec<double>::mdot(v, b.n, 0, v, b.partial, b.red + 2 * kRedStride, s));
    double h[kRedStride];
    CSD_HIP(hipMemcpyAsync(h, b.red + 2 * kRedStride, sizeof(h), hipMemcpyDeviceToHost, s));
    CSD_HIP(hipStreamSynchronize(s));
    out = std::sqrt(h[kRedStride - 1]);
    return CSDYN_OK;
}

static int32_t project_p(BShell &b, double *v, hipStream_t s) {
    const int64_t ncell = b.n / 4;
    CSD_TRY(Vec<double>::pmoments(v, b.ctx->dg.vol, ncell, b.partial, b.red + 2 * kRedStride, s));
    double h[kRedStride];
    CSD_HIP(hipMemcpyAsync(h, b.red + 2 * kRedStride, sizeof(h), hipMemcpyDeviceToHost, s));
    CSD_HIP(hipStreamSynchronize(s));
    return Vec<double>::padd(v, ncell, -h[0] / h[1], s);
}

struct ShellState {
    double beta0 = 0, beta = 0, bnorm = 0, tol = 0, est = 0;
    int iters = 0, restarts = 0, jdone = 0;
    bool conv = false, live = false;
    std::vector<double> H, cs, sn, g, y;
};

static int32_t residual(BShell &b, const double *x, hipStream_t s) {
    CSD_TRY(op_launch(b.ctx, x, b.tmp, s));
    CSD_TRY(Vec<double>::copy(b.r, b.bproj, b.n, s));
    return Vec<double>::axpby(-1.0, b.tmp, 1.0, b.r, b.n, s);
}

static int32_t batch_solve(csdyn_batch *bt, const double *const *bs, double *const *xs, bool use_graph,
                           hipStream_t s0, csdyn_gmres_stats *stats) {
    const int ns = bt->nshell, m = bt->m;
    const csdyn_gmres_opts &o = bt->o;
    std::vector<ShellState> S(ns);
    for (int i = 0; i < ns; ++i) {
        BShell &b = bt->sh[i];
        ShellState &q = S[i];
        q.H.assign(size_t(m + 1) * m, 0.0);
        q.cs.assign(m, 0.0);
        q.sn.assign(m, 0.0);
        q.g.assign(m + 1, 0.0);
        q.y.assign(m, 0.0);
        CSD_TRY(Vec<double>::copy(b.bproj, bs[i], b.n, s0));
        if (b.ctx->op.kind == CSDYN_VP) CSD_TRY(project_p(b, b.bproj, s0));
        CSD_TRY(residual(b, xs[i], s0));
        CSD_TRY(dev_norm(b, b.r, q.beta0, s0));
        if (!std::isfinite(q.beta0)) { set_error("batch: shell %d: non-finite initial residual", i); return CSDYN_EBREAKDOWN; }
        q.bnorm = q.beta0;
        if (o.rhs_relative) CSD_TRY(dev_norm(b, b.bproj, q.bnorm, s0));
        q.tol = std::max(o.atol, o.rtol * (o.rhs_relative ? q.bnorm : q.beta0));
        q.beta = q.est = q.beta0;
        q.conv = q.beta0 <= q.tol;
    }
    for (;;) {
        uint64_t cyc = 0;
        for (int i = 0; i < ns; ++i)
            if (!S[i].conv && S[i].iters < o.maxit) cyc |= uint64_t(1) << i;
        if (!cyc) break;
        for (int i = 0; i < ns; ++i) {
            if (!(cyc >> i & 1)) continue;
            BShell &b = bt->sh[i];
            ShellState &q = S[i];
            CSD_TRY(Vec<double>::copy(b.V, b.r, b.n, s0));
            CSD_TRY(Vec<double>::scale(b.V, b.n, 1.0 / q.beta, s0));
            std::fill(q.g.begin(), q.g.end(), 0.0);
            q.g[0] = q.beta;
            q.jdone = 0;
            q.live = true;
        }
        // the steps run on the batch's own stream (capture is not possible on the
        // legacy default stream), after everything issued so far on s0
        hipStream_t so = bt->origin;
        CSD_HIP(hipEventRecord(bt->ready, s0));
        CSD_HIP(hipStreamWaitEvent(so, bt->ready, 0));
        for (int j = 0; j < m; ++j) {
            uint64_t act = 0;
            for (int i = 0; i < ns; ++i)
                if ((cyc >> i & 1) && S[i].live) act |= uint64_t(1) << i;
            if (!act) break;
            if (use_graph) {
                hipGraphExec_t ex;
                CSD_TRY(graph_for(bt, act, j, so, ex));
                CSD_HIP(hipGraphLaunch(ex, so));
            } else {
                CSD_TRY(issue_step(bt, act, j, so));
            }
            CSD_HIP(hipStreamSynchronize(so));
            for (int i = 0; i < ns; ++i) {
                if (!(act >> i & 1)) continue;
                ShellState &q = S[i];
                const double *h1 = bt->hred + size_t(i) * 2 * kRedStride;
                for (int k = 0; k <= j; ++k) q.H[size_t(k) * m + j] = h1[k];
                const double ww = h1[kRedStride - 1], nn = h1[2 * kRedStride - 1];
                const double hn = std::sqrt(std::max(nn, 0.0));
                q.H[size_t(j + 1) * m + j] = hn;
                q.iters += 1;
                q.jdone = j + 1;
                if (!std::isfinite(hn) || !std::isfinite(ww)) {
                    set_error("batch: shell %d: non-finite Arnoldi vector", i);
                    return CSDYN_EBREAKDOWN;
                }
                for (int k = 0; k < j; ++k) {
                    const double a = q.H[size_t(k) * m + j], c = q.H[size_t(k + 1) * m + j];
                    q.H[size_t(k) * m + j] = q.cs[k] * a + q.sn[k] * c;
                    q.H[size_t(k + 1) * m + j] = -q.sn[k] * a + q.cs[k] * c;
                }
                const double a = q.H[size_t(j) * m + j], c = q.H[size_t(j + 1) * m + j];
                const double den = std::hypot(a, c);
                q.cs[j] = a / den;
                q.sn[j] = c / den;
                q.H[size_t(j) * m + j] = den;
                q.H[size_t(j + 1) * m + j] = 0.0;
                q.g[j + 1] = -q.sn[j] * q.g[j];
                q.g[j] = q.cs[j] * q.g[j];
                q.est = std::fabs(q.g[j + 1]);
                const bool happy = hn <= 1e-14 * std::sqrt(ww);
                if (q.est <= q.tol || happy) q.conv = true;
                if (q.conv || q.iters >= o.maxit) q.live = false;
            }
        }
        for (int i = 0; i < ns; ++i) {
            if (!(cyc >> i & 1)) continue;
            BShell &b = bt->sh[i];
            ShellState &q = S[i];
            const int jd = q.jdone;
            for (int k = jd - 1; k >= 0; --k) {
                double acc = q.g[k];
                for (int l = k + 1; l < jd; ++l) acc -= q.H[size_t(k) * m + l] * q.y[l];
                q.y[k] = acc / q.H[size_t(k) * m + k];
            }
            CSD_TRY(Vec<double>::lincomb(xs[i], b.Z, b.n, jd, q.y.data(), s0));
            CSD_TRY(residual(b, xs[i], s0));
            CSD_TRY(dev_norm(b, b.r, q.beta, s0));
            if (!q.conv) q.restarts += 1;
        }
    }
    int32_t rc = CSDYN_OK;
    for (int i = 0; i < ns; ++i) {
        BShell &b = bt->sh[i];
        if (b.ctx->op.kind == CSDYN_VP) CSD_TRY(project_p(b, xs[i], s0));
        if (!S[i].conv) rc = CSDYN_ENOTCONV;
        if (stats) {
            csdyn_gmres_stats &st = stats[i];
            std::memset(&st, 0, sizeof(st));
            st.iters = S[i].iters;
            st.restarts = S[i].restarts;
            st.relres_true = S[i].beta0 > 0 ? S[i].beta / S[i].beta0 : 0.0;
            st.relres_est = S[i].beta0 > 0 ? S[i].est / S[i].beta0 : 0.0;
            st.res0 = S[i].beta0;
            st.res_true = S[i].beta;
            st.bnorm = S[i].bnorm;
        }
    }
    CSD_HIP(hipStreamSynchronize(s0));
    return rc;
}

}  // namespace csd

using namespace csd;

extern "C" int32_t csdyn_batch_workspace_bytes(int32_t nshell, const csdyn_opctx *const *ops,
                                               const csdyn_gmres_opts *o, size_t *bytes) {
    clear_error();
    CSD_TRY(check_batch(nshell, ops, nullptr, o));
    if (!bytes) { set_error("batch: null bytes"); return CSDYN_EINVAL; }
    *bytes = batch_bytes(nshell, ops, o->restart);
    return CSDYN_OK;
}

extern "C" int32_t csdyn_batch_setup(int32_t nshell, const csdyn_opctx *const *ops, const csdyn_ras *const *pcs,
                                     const csdyn_gmres_opts *o, void *ws, size_t ws_bytes, csdyn_batch **out) {
    clear_error();
    CSD_TRY(check_batch(nshell, ops, pcs, o));
    if (!ws || !out) { set_error("batch: null workspace or output"); return CSDYN_EINVAL; }
    const size_t need = batch_bytes(nshell, ops, o->restart);
    if (ws_bytes < need) { set_error("batch: workspace %zu < %zu bytes", ws_bytes, need); return CSDYN_ENOMEM; }
    std::unique_ptr<csdyn_batch> bt(new csdyn_batch);
    bt->nshell = nshell;
    bt->m = o->restart;
    bt->o = *o;
    bt->sh.resize(nshell);
    Carver c(ws);
    for (int i = 0; i < nshell; ++i) {
        BShell &b = bt->sh[i];
        b.ctx = ops[i];
        b.pc = pcs ? pcs[i] : nullptr;
        b.n = 24 * int64_t(ops[i]->g.n) * ops[i]->g.n * ops[i]->g.nr;
        carve_shell(c, b, bt->m);
        CSD_HIP(hipStreamCreateWithFlags(&b.st, hipStreamNonBlocking));
        CSD_HIP(hipEventCreateWithFlags(&b.join, hipEventDisableTiming));
    }
    CSD_HIP(hipEventCreateWithFlags(&bt->fork, hipEventDisableTiming));
    CSD_HIP(hipEventCreateWithFlags(&bt->ready, hipEventDisableTiming));
    CSD_HIP(hipStreamCreateWithFlags(&bt->origin, hipStreamNonBlocking));
    CSD_HIP(hipHostMalloc((void **)&bt->hred, sizeof(double) * 2 * kRedStride * nshell, hipHostMallocDefault));
    *out = bt.release();
    return CSDYN_OK;
}

extern "C" int32_t csdyn_gmres_solve_batched(csdyn_batch *bt, const double *const *b, double *const *x,
                                             int32_t use_graph, void *stream, csdyn_gmres_stats *stats) {
    clear_error();
    if (!bt || !b || !x) { set_error("batch: null argument"); return CSDYN_EINVAL; }
    for (int i = 0; i < bt->nshell; ++i)
        if (!b[i] || !x[i]) { set_error("batch: null vector for shell %d", i); return CSDYN_EINVAL; }
    return batch_solve(bt, b, x, use_graph != 0, (hipStream_t)stream, stats);
}

extern "C" void csdyn_batch_destroy(csdyn_batch *bt) { delete bt; }
