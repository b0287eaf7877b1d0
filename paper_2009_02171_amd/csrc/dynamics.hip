// The explicit parts of the semi-implicit time step (Sec. 3.1): the nonlinear
// terms f1 = -(u.grad)u + (1/(E Pm)) (B.grad)B and f3 = (B.grad)u - (u.grad)B
// (eq. nonlinearoperator), the Crank-Nicolson right-hand side of Step 1 with
// the Adams-Bashforth combination of the nonlinear terms (eqs. tsvelocity,
// tsmag), and the Step-3 state (u^{n+1}, P^{n+1}) the next step starts from.
//
// (a.grad)b is taken in the conservative form div(a b_c) of each Cartesian
// component c (Sec. 3.2, eq. nonlinearint; the vectors are stored in Cartesian
// components, whose Christoffel source terms vanish): the finite-volume sum
// over a cell's six faces of (a_f . sqrt(g) g^m) (b_c)_f times the face area,
// over the cell volume, with a_f, b_f the means of the two cells' values (the
// neighbour beyond a panel edge is its ghost, beyond a wall the wall ghost of
// the field's own system), and through a panel-edge face the mean of the two
// panels' one-sided fluxes, so each component is exactly conserved.
#include "op_dev.h"
#include "profile.h"

namespace csd {
namespace {

// Value of field x at a face neighbour of cell (p, i, j, k): the cell itself
// inside the panel, the ghost beyond a panel edge (G), the wall ghost of
// system `kind` beyond a wall.
__device__ __forceinline__ V4<double> ext_val(const DevGeom &g, const double *x, const double *G, int kind, int p,
                                              int i, int j, int k) {
    if (k < 0 || k >= g.nr) {
        const int kin = k < 0 ? 0 : g.nr - 1;
        const V4<double> xin = ld4(x + 4 * cell_ix(g.n, g.nr, p, i, j, kin));
        const double *nv = g.nrm + ((size_t(p) * g.n + j) * g.n + i) * 3;
        const double nvv[3] = {nv[0], nv[1], nv[2]};
        return wall_ghost(xin, kind, nvv, k < 0 ? g.wq2_bot : g.wq2_top);
    }
    return fetch_ext(g, x, G, p, i, j, k);
}

// The advective products through one face, with outward face vector s
// (sqrt(g) g^m times the cell's weight): [0] (u.s) u_f, [1] (B.s) B_f,
// [2] (B.s) u_f, [3] (u.s) B_f; each accumulated with weight w; with the
// temperature, also (u.s) Theta_f into *ath.
__device__ __forceinline__ void face_products(const V4<double> &uc, const V4<double> &un, const V4<double> &Bc,
                                              const V4<double> &Bn, const double s[3], double w,
                                              double acc[4][3], double th_f, double *ath) {
    double uf[3], Bf[3];
    for (int d = 0; d < 3; ++d) {
        uf[d] = 0.5 * (uc.c[d] + un.c[d]);
        Bf[d] = 0.5 * (Bc.c[d] + Bn.c[d]);
    }
    const double Fu = w * (s[0] * uf[0] + s[1] * uf[1] + s[2] * uf[2]);
    const double FB = w * (s[0] * Bf[0] + s[1] * Bf[1] + s[2] * Bf[2]);
    for (int d = 0; d < 3; ++d) {
        acc[0][d] += Fu * uf[d];
        acc[1][d] += FB * Bf[d];
        acc[2][d] += FB * uf[d];
        acc[3][d] += Fu * Bf[d];
    }
    if (ath) *ath += Fu * th_f;
}

// Theta at the cell and its face neighbour (isothermal walls); 0 without T.
__device__ __forceinline__ double theta_face(const DevGeom &g, const double *T, const double *GT, int p, int i, int j,
                                             int k, int ni, int nj, int nk) {
    if (!T) return 0.0;
    const double tc = T[4 * cell_ix(g.n, g.nr, p, i, j, k) + 3];
    return 0.5 * (tc + ext_val(g, T, GT, CSDYN_VT, p, ni, nj, nk).c[3]);
}

// One-sided products through lateral face f (0 W, 1 E, 2 S, 3 N) of cell
// (p, i, j, k), from panel p's own values, weight w.
__device__ void lateral_face(const DevGeom &g, const double *u, const double *Gu, const double *B, const double *GB,
                             const double *T, const double *GT, int p, int i, int j, int k, int f, double w,
                             double acc[4][3], double *ath) {
    const int n = g.n;
    const size_t nf = size_t(n) * (n + 1);
    int ni = i, nj = j;
    const double *tv;
    if (f <= 1) {
        ni = f == 0 ? i - 1 : i + 1;
        tv = g.t1 + (p * nf + size_t(j) * (n + 1) + (f == 0 ? i : i + 1)) * 3;
    } else {
        nj = f == 2 ? j - 1 : j + 1;
        tv = g.t2 + (p * nf + size_t(f == 2 ? j : j + 1) * n + i) * 3;
    }
    const double sg = (f == 1 || f == 3) ? 1.0 : -1.0;
    const double s[3] = {sg * tv[0], sg * tv[1], sg * tv[2]};
    const V4<double> uc = ld4(u + 4 * cell_ix(n, g.nr, p, i, j, k));
    const V4<double> Bc = ld4(B + 4 * cell_ix(n, g.nr, p, i, j, k));
    const V4<double> un = ext_val(g, u, Gu, CSDYN_VP, p, ni, nj, k);
    const V4<double> Bn = ext_val(g, B, GB, CSDYN_BP, p, ni, nj, k);
    face_products(uc, un, Bc, Bn, s, w, acc, theta_face(g, T, GT, p, i, j, k, ni, nj, k), ath);
}

// f1 = -(u.grad)u + cB (B.grad)B, f3 = (B.grad)u - (u.grad)B on every cell;
// with the velocity-temperature state T, f1's scalar slot = -(u.grad)Theta
// (f2), else 0.
__global__ void k_nonlinear(DevGeom g, const double *__restrict__ u, const double *__restrict__ Gu,
                            const double *__restrict__ B, const double *__restrict__ GB,
                            const double *__restrict__ T, const double *__restrict__ GT, double cB,
                            double *__restrict__ f1, double *__restrict__ f3) {
    const int n = g.n, nr = g.nr;
    const int64_t ncell = 6 * int64_t(n) * n * nr;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int i = int(c % n), j = int((c / n) % n), k = int((c / (int64_t(n) * n)) % nr);
    const int p = int(c / (int64_t(n) * n * nr));
    const double rk = g.rk[k];
    const double wl = g.isc[size_t(j) * n + i] / rk;  // lateral faces: (t . a_f) b_f / (r_k sqrt(g)/r^2 h_s)
    double acc[4][3] = {}, th = 0.0;
    double *ath = T ? &th : nullptr;
    for (int f = 0; f < 4; ++f) {
        const bool seam = (f == 0 && i == 0) || (f == 1 && i == n - 1) || (f == 2 && j == 0) || (f == 3 && j == n - 1);
        if (!seam) {
            lateral_face(g, u, Gu, B, GB, T, GT, p, i, j, k, f, wl, acc, ath);
            continue;
        }
        // mean of this panel's and the neighbour panel's one-sided outward fluxes
        lateral_face(g, u, Gu, B, GB, T, GT, p, i, j, k, f, 0.5 * wl, acc, ath);
        const int a = (p * 4 + f) * n + (f <= 1 ? j : i);
        const int q = g.fc[4 * a], eq = g.fc[4 * a + 1], tq = g.fc[4 * a + 2];
        const int iq = eq == 0 ? 0 : eq == 1 ? n - 1 : tq, jq = eq == 2 ? 0 : eq == 3 ? n - 1 : tq;
        lateral_face(g, u, Gu, B, GB, T, GT, q, iq, jq, k, eq, -0.5 * wl, acc, ath);
    }
    // radial faces: sqrt(g) g^3 = r_f^2 (sqrt(g)/r^2) r_hat
    const double *nv = g.nrm + ((size_t(p) * n + j) * n + i) * 3;
    const V4<double> uc = ld4(u + 4 * c), Bc = ld4(B + 4 * c);
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        const double rf = g.rf[k + (sgn > 0 ? 1 : 0)];
        const double wr = sgn * rf * rf / (rk * rk * g.hr);
        const V4<double> un = ext_val(g, u, Gu, CSDYN_VP, p, i, j, k + sgn);
        const V4<double> Bn = ext_val(g, B, GB, CSDYN_BP, p, i, j, k + sgn);
        const double s[3] = {nv[0], nv[1], nv[2]};
        face_products(uc, un, Bc, Bn, s, wr, acc, theta_face(g, T, GT, p, i, j, k, i, j, k + sgn), ath);
    }
    for (int d = 0; d < 3; ++d) {
        f1[4 * c + d] = -acc[0][d] + cB * acc[1][d];
        f3[4 * c + d] = acc[2][d] - acc[3][d];
    }
    f1[4 * c + 3] = -th;
    f3[4 * c + 3] = 0.0;
}

__global__ void k_ghost_fill(DevGeom g, const double *__restrict__ x, double *__restrict__ G) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < g.n) ghost_at(g, x, G, int(blockIdx.z), int(blockIdx.y), t);
}

// rhs = 2 xhat - rhs + c1 fn + c2 fm + c3 gf, where rhs holds A xhat on entry;
// the scalar slot set to 0 unless keep_scalar (the VT system's Theta row).
__global__ void k_cn_combine(const double *__restrict__ xhat, const double *__restrict__ fn,
                             const double *__restrict__ fm, const double *__restrict__ gf, double c1, double c2,
                             double c3, double *__restrict__ rhs, int64_t ncell, int keep_scalar) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < 4 * ncell; e += stride) {
        if ((e & 3) == 3 && !keep_scalar) {
            rhs[e] = 0.0;
            continue;
        }
        double v = 2.0 * xhat[e] - rhs[e] + c1 * fn[e];
        if (fm) v += c2 * fm[e];
        if (gf) v += c3 * gf[e];
        rhs[e] = v;
    }
}

// out_3 = 0 (the vector rows of A x alone)
__global__ void k_zero_scalar(double *__restrict__ out, int64_t ncell) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < ncell; c += stride) out[4 * c + 3] = 0.0;
}

// out_3 = x_3 (the state keeps the solve's pressure next to the corrected vector)
__global__ void k_keep_scalar(const double *__restrict__ x, double *__restrict__ out, int64_t ncell) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < ncell; c += stride)
        out[4 * c + 3] = x[4 * c + 3];
}

dim3 grid_for(int64_t n) { return dim3(unsigned(n > 0 ? (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192 : 1)); }

bool same_grid(const csdyn_opctx *a, const csdyn_opctx *b) {
    return a->g.n == b->g.n && a->g.nr == b->g.nr && a->g.ri == b->g.ri && a->g.ro == b->g.ro;
}

bool overlaps(const void *a, const void *b, size_t bytes) {
    const char *x = static_cast<const char *>(a), *y = static_cast<const char *>(b);
    return x < y + bytes && y < x + bytes;
}

}  // namespace
}  // namespace csd

using namespace csd;

extern "C" int32_t csdyn_nonlinear_workspace_bytes(const csdyn_opctx *ctx, size_t *bytes) {
    clear_error();
    if (!ctx || !bytes) { set_error("nonlinear: null argument"); return CSDYN_EINVAL; }
    Carver c(nullptr);
    for (int q = 0; q < 3; ++q) c.take<double>(size_t(96) * ctx->g.n * ctx->g.nr);
    *bytes = c.off + 256;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_nonlinear(const csdyn_opctx *vp, const csdyn_opctx *bp, const double *u, const double *B,
                                   const double *T, double cB, double *f1, double *f3, void *ws, size_t ws_bytes,
                                   void *stream) {
    clear_error();
    if (!vp || !bp || !u || !B || !f1 || !f3 || !ws) { set_error("nonlinear: null argument"); return CSDYN_EINVAL; }
    if (vp->op.kind != CSDYN_VP || bp->op.kind != CSDYN_BP) {
        set_error("nonlinear: vp must be a velocity-pressure context and bp a magnetic one");
        return CSDYN_EINVAL;
    }
    if (!same_grid(vp, bp)) { set_error("nonlinear: the two contexts have different grids"); return CSDYN_EINVAL; }
    const int n = vp->g.n, nr = vp->g.nr;
    const int64_t ncell = 6 * int64_t(n) * n * nr;
    const size_t vb = size_t(4) * ncell * sizeof(double);
    if (f1 == f3 || overlaps(f1, f3, vb) || overlaps(f1, u, vb) || overlaps(f1, B, vb) || overlaps(f3, u, vb) ||
        overlaps(f3, B, vb) || (T && (overlaps(f1, T, vb) || overlaps(f3, T, vb)))) {
        set_error("nonlinear: f1 and f3 must not alias each other or the inputs");
        return CSDYN_EINVAL;
    }
    Carver c(ws);
    double *Gu = c.take<double>(size_t(96) * n * nr), *GB = c.take<double>(size_t(96) * n * nr);
    double *GT = c.take<double>(size_t(96) * n * nr);
    if (c.off + 256 > ws_bytes) { set_error("nonlinear: workspace %zu < %zu bytes", ws_bytes, c.off + 256); return CSDYN_ENOMEM; }
    hipStream_t s = (hipStream_t)stream;
    const DevGeom &g = vp->dg;
    const dim3 eb(64), eg((n + 63) / 64, nr, 24);
    {
        ProfScope ps("nl_ghosts", ncell, (T ? 3.0 : 2.0) * 24 * n * nr * 5 * 4 * sizeof(double), s);
        hipLaunchKernelGGL(k_ghost_fill, eg, eb, 0, s, g, u, Gu);
        hipLaunchKernelGGL(k_ghost_fill, eg, eb, 0, s, g, B, GB);
        if (T) hipLaunchKernelGGL(k_ghost_fill, eg, eb, 0, s, g, T, GT);
        CSD_HIP(hipGetLastError());
    }
    // u and B (and T) read once, f1 and f3 written once
    ProfScope ps("nonlinear", ncell, (T ? 5.0 : 4.0) * vb, s);
    hipLaunchKernelGGL(k_nonlinear, dim3(unsigned((ncell + 255) / 256)), dim3(256), 0, s, g, u, (const double *)Gu,
                       B, (const double *)GB, T, T ? (const double *)GT : nullptr, cB, f1, f3);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

extern "C" int32_t csdyn_cn_rhs(const csdyn_opctx *ctx, const double *xhat, const double *fn, const double *fm,
                                const double *gf, double c1, double c2, double c3, double *rhs, void *stream) {
    clear_error();
    if (!ctx || !xhat || !fn || !rhs) { set_error("cn_rhs: null argument"); return CSDYN_EINVAL; }
    if ((c2 != 0.0 && !fm) || (c3 != 0.0 && !gf)) { set_error("cn_rhs: a term with a nonzero coefficient has no vector"); return CSDYN_EINVAL; }
    const int64_t ncell = 6 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr;
    const size_t vb = size_t(4) * ncell * sizeof(double);
    if (overlaps(rhs, xhat, vb) || overlaps(rhs, fn, vb) || (fm && overlaps(rhs, fm, vb)) || (gf && overlaps(rhs, gf, vb))) {
        set_error("cn_rhs: rhs must not alias an input");
        return CSDYN_EINVAL;
    }
    hipStream_t s = (hipStream_t)stream;
    CSD_TRY(op_launch(ctx, xhat, rhs, s));
    hipLaunchKernelGGL(k_cn_combine, grid_for(4 * ncell), dim3(256), 0, s, xhat, fn, c2 != 0.0 ? fm : nullptr,
                       c3 != 0.0 ? gf : nullptr, c1, c2, c3, rhs, ncell, int(ctx->op.kind == CSDYN_VT));
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

extern "C" int32_t csdyn_step3_state(const csdyn_opctx *ctx, const double *x, double *state, void *stream) {
    clear_error();
    CSD_TRY(csdyn_project(ctx, x, state, stream));
    const int64_t ncell = 6 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr;
    hipLaunchKernelGGL(k_keep_scalar, grid_for(ncell), dim3(256), 0, (hipStream_t)stream, x, state, ncell);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

extern "C" int32_t csdyn_vector_rows(const csdyn_opctx *ctx, const double *x, double *y, void *stream) {
    clear_error();
    if (!ctx || !x || !y) { set_error("vector_rows: null argument"); return CSDYN_EINVAL; }
    if (ctx->op.kind == CSDYN_VT) { set_error("vector_rows: the VT system's vector rows read its scalar part"); return CSDYN_EINVAL; }
    const int64_t ncell = 6 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr;
    if (overlaps(x, y, size_t(4) * ncell * sizeof(double))) { set_error("vector_rows: x and y alias"); return CSDYN_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    CSD_TRY(op_launch(ctx, x, y, s));
    hipLaunchKernelGGL(k_zero_scalar, grid_for(ncell), dim3(256), 0, s, y, ncell);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}
