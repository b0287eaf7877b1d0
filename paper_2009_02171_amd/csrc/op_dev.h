// Device code of the finite-volume operator (Sec. 3.2, eq. divdiscretization),
// shared by the operator's own kernels (op.hip) and the persistent batched
// Arnoldi step (batched.hip): vector helpers, ghost values beyond panel edges,
// the averaged edge-face fluxes, wall ghosts and the stencil's layer march.
#pragma once

#include <type_traits>

#include "common.h"

namespace csd {

template <class T>
struct V4 {
    T c[4];
};

template <class T>
__device__ __forceinline__ V4<T> ld4(const T *p) {
    V4<T> v;
    if constexpr (sizeof(T) == 8) {
        const double2 a = reinterpret_cast<const double2 *>(p)[0];
        const double2 b = reinterpret_cast<const double2 *>(p)[1];
        v.c[0] = a.x; v.c[1] = a.y; v.c[2] = b.x; v.c[3] = b.y;
    } else {
        const float4 a = *reinterpret_cast<const float4 *>(p);
        v.c[0] = a.x; v.c[1] = a.y; v.c[2] = a.z; v.c[3] = a.w;
    }
    return v;
}

template <class T>
__device__ __forceinline__ void st4(T *p, const V4<T> &v) {
    if constexpr (sizeof(T) == 8) {
        reinterpret_cast<double2 *>(p)[0] = make_double2(v.c[0], v.c[1]);
        reinterpret_cast<double2 *>(p)[1] = make_double2(v.c[2], v.c[3]);
    } else {
        *reinterpret_cast<float4 *>(p) = make_float4(v.c[0], v.c[1], v.c[2], v.c[3]);
    }
}

__device__ __forceinline__ int64_t cell_ix(int n, int nr, int p, int i, int j, int k) {
    return ((int64_t(p) * nr + k) * n + j) * n + i;
}

__device__ __forceinline__ int64_t ghost_ix(int n, int nr, int p, int e, int k, int t) {
    return ((int64_t(p * 4 + e) * nr + k) * n + t);
}

// Edge-flux buffer: the 4 averaged Laplacian fluxes of face (p, e, k, t) at
// 4 * ghost_ix, then the divergence fluxes, their tangential index padded to
// a multiple of 4 so that four neighbouring faces are one aligned load.
__device__ __forceinline__ int64_t fdiv_ix(int n, int nr, int p, int e, int k, int t) {
    return int64_t(24) * nr * n * 4 + (int64_t(p * 4 + e) * nr + k) * ((n + 3) & ~3) + t;
}

// Value at an extended position of panel X (one cell beyond an edge: the
// ghost; both beyond: the cube-corner rule f(-1,0) + f(0,-1) - f(0,0)).
template <class T>
__device__ V4<T> fetch_ext(const DevGeom &g, const T *x, const T *G, int X, int i, int j, int k) {
    const int n = g.n, nr = g.nr;
    const bool iin = i >= 0 && i < n, jin = j >= 0 && j < n;
    if (iin && jin) return ld4(x + 4 * cell_ix(n, nr, X, i, j, k));
    if (!iin && !jin) {
        const int ic = i < 0 ? 0 : n - 1, jc = j < 0 ? 0 : n - 1;
        V4<T> a = ld4(G + 4 * ghost_ix(n, nr, X, i < 0 ? 0 : 1, k, jc));
        V4<T> b = ld4(G + 4 * ghost_ix(n, nr, X, j < 0 ? 2 : 3, k, ic));
        V4<T> c = ld4(x + 4 * cell_ix(n, nr, X, ic, jc, k));
        V4<T> r;
        for (int q = 0; q < 4; ++q) r.c[q] = a.c[q] + b.c[q] - c.c[q];
        return r;
    }
    if (!iin) return ld4(G + 4 * ghost_ix(n, nr, X, i < 0 ? 0 : 1, k, j));
    return ld4(G + 4 * ghost_ix(n, nr, X, j < 0 ? 2 : 3, k, i));
}

// Ghost value one cell beyond panel edge pe % 4 of panel pe / 4, plane k,
// tangential index t < n.
template <class T>
__device__ __forceinline__ void ghost_at(const DevGeom &g, const T *__restrict__ x, T *__restrict__ G, int pe, int k,
                                         int t) {
    const int n = g.n, nr = g.nr;
    const int a = pe * n + t;
    const int q = g.gh_i[4 * a], fix = g.gh_i[4 * a + 1], idx = g.gh_i[4 * a + 2], m0 = g.gh_i[4 * a + 3];
    V4<T> acc = {};
    for (int m = 0; m < 4; ++m) {
        const T w = T(g.gh_w[4 * a + m]);
        const int64_t c = fix ? cell_ix(n, nr, q, idx, m0 + m, k) : cell_ix(n, nr, q, m0 + m, idx, k);
        const V4<T> v = ld4(x + 4 * c);
        for (int s = 0; s < 4; ++s) acc.c[s] += w * v.c[s];
    }
    st4(G + 4 * ghost_ix(n, nr, pe / 4, pe % 4, k, t), acc);
}

// One-sided outward fluxes of panel X's first-layer cell at edge e,
// tangential index t, plane k, from X's own extended values:
// out[0..3] Laplacian flux sqrt(g) g^{mn} d_n f of each component,
// out[4] divergence flux (sqrt(g) g^m / r) . (v_c + v_nb)/2.
template <class T>
__device__ void one_sided(const DevGeom &g, const T *x, const T *G, int X, int e, int t, int k, T out[5]) {
    const int n = g.n;
    const size_t nf = size_t(n) * (n + 1);
    const T ih = T(1.0 / g.hs), i4h = T(0.25 / g.hs);
    if (e <= 1) {
        const int j = t, fi = e == 0 ? 0 : n, il = fi - 1, ir = fi;
        const size_t a = size_t(j) * (n + 1) + fi;
        const T a11 = T(g.a11x[a]), a12 = T(g.a12x[a]);
        const V4<T> fl = fetch_ext(g, x, G, X, il, j, k), fr = fetch_ext(g, x, G, X, ir, j, k);
        const V4<T> flp = fetch_ext(g, x, G, X, il, j + 1, k), frp = fetch_ext(g, x, G, X, ir, j + 1, k);
        const V4<T> flm = fetch_ext(g, x, G, X, il, j - 1, k), frm = fetch_ext(g, x, G, X, ir, j - 1, k);
        const T sg = e == 1 ? T(1) : T(-1);
        for (int c = 0; c < 4; ++c)
            out[c] = sg * (a11 * (fr.c[c] - fl.c[c]) * ih + a12 * (flp.c[c] + frp.c[c] - flm.c[c] - frm.c[c]) * i4h);
        const double *tv = g.t1 + (X * nf + a) * 3;
        out[4] = sg * T(0.5) * (T(tv[0]) * (fl.c[0] + fr.c[0]) + T(tv[1]) * (fl.c[1] + fr.c[1]) + T(tv[2]) * (fl.c[2] + fr.c[2]));
    } else {
        const int i = t, fj = e == 2 ? 0 : n, jl = fj - 1, jr = fj;
        const size_t a = size_t(fj) * n + i;
        const T a22 = T(g.a22y[a]), a12 = T(g.a12y[a]);
        const V4<T> fl = fetch_ext(g, x, G, X, i, jl, k), fr = fetch_ext(g, x, G, X, i, jr, k);
        const V4<T> fpl = fetch_ext(g, x, G, X, i + 1, jl, k), fpr = fetch_ext(g, x, G, X, i + 1, jr, k);
        const V4<T> fml = fetch_ext(g, x, G, X, i - 1, jl, k), fmr = fetch_ext(g, x, G, X, i - 1, jr, k);
        const T sg = e == 3 ? T(1) : T(-1);
        for (int c = 0; c < 4; ++c)
            out[c] = sg * (a22 * (fr.c[c] - fl.c[c]) * ih + a12 * (fpl.c[c] + fpr.c[c] - fml.c[c] - fmr.c[c]) * i4h);
        const double *tv = g.t2 + (X * nf + a) * 3;
        out[4] = sg * T(0.5) * (T(tv[0]) * (fl.c[0] + fr.c[0]) + T(tv[1]) * (fl.c[1] + fr.c[1]) + T(tv[2]) * (fl.c[2] + fr.c[2]));
    }
}

// Averaged flux records of panel-edge face (pe, k, t), t < n.
template <class T>
__device__ __forceinline__ void edgeflux_at(const DevGeom &g, const T *__restrict__ x, const T *__restrict__ G,
                                            T *__restrict__ SF, int pe, int k, int t) {
    const int n = g.n, nr = g.nr;
    const int p = pe / 4, e = pe % 4;
    T oa[5], ob[5];
    one_sided(g, x, G, p, e, t, k, oa);
    const int a = pe * n + t;
    one_sided(g, x, G, g.fc[4 * a], g.fc[4 * a + 1], g.fc[4 * a + 2], k, ob);
    T *o = SF + 4 * ghost_ix(n, nr, p, e, k, t);
    for (int c = 0; c < 4; ++c) o[c] = T(0.5) * (oa[c] - ob[c]);
    SF[fdiv_ix(n, nr, p, e, k, t)] = T(0.5) * (oa[4] - ob[4]);
}

struct RowCoef {
    int kind;      // CSDYN_VP, CSDYN_BP or CSDYN_VT
    double c_lap;  // dt*E (VP, VT) or dt*E/Pm (BP)
    double c_cor;  // 2 dt (VP, VT), 0 (BP)
    double dt;
    double c_th;   // VT: dt*E/Pr (the Theta Laplacian)
    double c_r1;   // VT: dt*Ra/r_o (buoyancy: times r Theta r_hat)
    double c_r2;   // VT: dt*E*r_i*r_o (times (r_hat . u) / r^2)
};

// Wall ghost of a boundary cell (no-slip u, Neumann P; pseudo-vacuum B,
// Dirichlet P_b).  q = (r_in / r_ghost)^2.
template <class T>
__device__ __forceinline__ V4<T> wall_ghost(const V4<T> &xin, int kind, const T nv[3], T q) {
    V4<T> gv;
    if (kind == CSDYN_VP) {
        gv.c[0] = -xin.c[0]; gv.c[1] = -xin.c[1]; gv.c[2] = -xin.c[2]; gv.c[3] = xin.c[3];
    } else if (kind == CSDYN_VT) {  // no-slip u, isothermal Theta
        gv.c[0] = -xin.c[0]; gv.c[1] = -xin.c[1]; gv.c[2] = -xin.c[2]; gv.c[3] = -xin.c[3];
    } else {
        const T nb = (T(1) + q) * (nv[0] * xin.c[0] + nv[1] * xin.c[1] + nv[2] * xin.c[2]);
        gv.c[0] = -xin.c[0] + nb * nv[0];
        gv.c[1] = -xin.c[1] + nb * nv[1];
        gv.c[2] = -xin.c[2] + nb * nv[2];
        gv.c[3] = -xin.c[3];
    }
    return gv;
}

// The stencil: one workgroup owns a TX x TY tile of columns of one panel and
// marches over a chunk of radial layers, one thread per column.  The halo of
// three layers sits in LDS (layer k for the lateral stencil, k+1 for the
// radial neighbour, k+2 being written) while layers k+3 and k+4 are in flight
// in registers; one barrier per layer, which orders LDS only so that the global
// loads stay in flight.  Every iteration issues the same loads in the same
// order (cells outside the panel read a zero page), so the compiler's
// in-order memory counters wait only for what a layer uses.  In tiles on a
// panel edge the averaged edge-face fluxes travel with the layers through LDS,
// requested by threads that have no border cell, so they hold no registers.
constexpr int kMaxChunk = 64;  // radial layers per workgroup

// Workgroup barrier that orders LDS only (__syncthreads would also wait for
// every global load in flight).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <class T>
struct Column {  // r-independent metric of one column (a11, a22 times 1/h, a12 times 1/(4h))
    T a11W, a11E, a12W, a12E, a22S, a22N, a12S, a12N, isc;
    T tW[3], tE[3], tS[3], tN[3], nv[3];
};

// LDS of one stencil workgroup: three halo layers [3][4][HC] (component-major),
// then for each of the three buffers the records of the tile's panel-edge
// faces: NF faces x 4 Laplacian fluxes, then NF divergence fluxes.  Face
// positions are fixed: W edge [0, TY), E edge [TY, 2TY), S edge
// [2TY, 2TY+TX), N edge [2TY+TX, NF).  Last, a slot per thread where
// threads without an extra record write it (never read).
template <int TX, int TY>
struct OpLds {
    static constexpr int HC = (TX + 2) * (TY + 2), NF = 2 * TY + 2 * TX, FA = 5 * NF;
    static constexpr int HALO = 3 * 4 * HC, DUMMY = HALO + 3 * FA, SIZE = DUMMY + 4 * TX * TY;
};

template <class T, int TX, int TY, bool EDGE, bool VT = false>
__device__ __forceinline__ void op_march(const DevGeom &g, const RowCoef &rc, int p, int bx, int by, int k0, int k1,
                                         const T *__restrict__ x, const T *__restrict__ G,
                                         const T *__restrict__ SF, T *__restrict__ y, T *lds, T (*layf)[8]) {
    using LL = OpLds<TX, TY>;
    constexpr int NT = TX * TY, HX = TX + 2, HY = TY + 2, HC = LL::HC, NRING = HC - NT, NF = LL::NF, FA = LL::FA;
    static_assert(NRING <= NT, "one border cell per thread");
    const int n = g.n, nr = g.nr;
    const int tx = threadIdx.x % TX, ty = threadIdx.x / TX;
    const int i = bx * TX + tx, j = by * TY + ty;
    const bool act = i < n && j < n;
    const int ic = min(i, n - 1), jc = min(j, n - 1);
    const size_t nf = size_t(n) * (n + 1);
    const int64_t kstride = int64_t(n) * n;
    const T *zp = reinterpret_cast<const T *>(g.zero);

    Column<T> m;
    {  // metric coefficients with the face-normal (1/h) and cross (1/(4h)) difference factors folded in
        const double ihd = 1.0 / g.hs, i4hd = 0.25 / g.hs;
        m.a11W = T(g.a11x[size_t(jc) * (n + 1) + ic] * ihd); m.a11E = T(g.a11x[size_t(jc) * (n + 1) + ic + 1] * ihd);
        m.a12W = T(g.a12x[size_t(jc) * (n + 1) + ic] * i4hd); m.a12E = T(g.a12x[size_t(jc) * (n + 1) + ic + 1] * i4hd);
        m.a22S = T(g.a22y[size_t(jc) * n + ic] * ihd); m.a22N = T(g.a22y[size_t(jc + 1) * n + ic] * ihd);
        m.a12S = T(g.a12y[size_t(jc) * n + ic] * i4hd); m.a12N = T(g.a12y[size_t(jc + 1) * n + ic] * i4hd);
    }
    m.isc = T(g.isc[size_t(jc) * n + ic]);
    for (int d = 0; d < 3; ++d) {
        m.tW[d] = T(g.t1[(p * nf + size_t(jc) * (n + 1) + ic) * 3 + d]);
        m.tE[d] = T(g.t1[(p * nf + size_t(jc) * (n + 1) + ic + 1) * 3 + d]);
        m.tS[d] = T(g.t2[(p * nf + size_t(jc) * n + ic) * 3 + d]);
        m.tN[d] = T(g.t2[(p * nf + size_t(jc + 1) * n + ic) * 3 + d]);
        m.nv[d] = T(g.nrm[((size_t(p) * n + jc) * n + ic) * 3 + d]);
    }
    const bool sW = i == 0, sE = i == n - 1, sS = j == 0, sN = j == n - 1;

    const T clap = T(rc.c_lap), ccor = T(rc.c_cor), cdt = T(rc.dt);

    // Every thread loads its own cell each layer and one more 4-value record:
    // a cell of the halo's border ring (threads r < NRING), else in edge
    // tiles a panel-edge face record: one request per face (its Laplacian
    // fluxes), then one per four faces (their divergence fluxes), edges in the
    // order W, E, S, N.  The records travel with the layer into LDS.
    auto source = [&](int hx, int hy, const T *&src, int64_t &step) {
        const int ii = bx * TX + hx - 1, jj = by * TY + hy - 1;
        const bool iin = ii >= 0 && ii < n, jin = jj >= 0 && jj < n;
        src = zp;
        step = 0;
        if (iin && jin) { src = x + 4 * cell_ix(n, nr, p, ii, jj, k0); step = 4 * kstride; }
        else if (jin && (ii == -1 || ii == n)) { src = G + 4 * ghost_ix(n, nr, p, ii < 0 ? 0 : 1, k0, jj); step = 4 * n; }
        else if (iin && (jj == -1 || jj == n)) { src = G + 4 * ghost_ix(n, nr, p, jj < 0 ? 2 : 3, k0, ii); step = 4 * n; }
    };
    const int r = threadIdx.x;
    const int own_h = (ty + 1) * HX + tx + 1;
    const T *own_src, *xsrc = zp;
    int64_t own_step, xstep = 0;
    source(tx + 1, ty + 1, own_src, own_step);
    // the extra record goes to lds[xoff + b * xbuf + c * xcomp] (buffer b)
    int xoff = LL::DUMMY + 4 * r, xbuf = 0, xcomp = 1;
    if (r < NRING) {
        int rhx, rhy;
        if (r < HX) { rhx = r; rhy = 0; }
        else if (r < 2 * HX) { rhx = r - HX; rhy = HY - 1; }
        else if (r < 2 * HX + HY - 2) { rhx = 0; rhy = 1 + r - 2 * HX; }
        else { rhx = HX - 1; rhy = 1 + r - 2 * HX - (HY - 2); }
        source(rhx, rhy, xsrc, xstep);
        xoff = rhy * HX + rhx;
        xbuf = 4 * HC;
        xcomp = HC;
    } else if (EDGE) {
        const bool eW = bx == 0, eE = (bx + 1) * TX >= n, eS = by == 0, eN = (by + 1) * TY >= n;
        const int cA = min(TY, n - by * TY), cB = min(TX, n - bx * TX);
        const int cnt[4] = {eW ? cA : 0, eE ? cA : 0, eS ? cB : 0, eN ? cB : 0};
        const int pos[4] = {0, TY, 2 * TY, 2 * TY + TX};
        const int q = r - NRING, nlap = cnt[0] + cnt[1] + cnt[2] + cnt[3];
        int lap_before = 0, div_before = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int t0 = e < 2 ? by * TY : bx * TX;
            const int nd = (cnt[e] + 3) / 4;
            const int ql = q - lap_before;  // Laplacian fluxes of face t0 + ql
            if (ql >= 0 && ql < cnt[e]) {
                xsrc = SF + 4 * ghost_ix(n, nr, p, e, k0, t0 + ql);
                xstep = 4 * int64_t(n);
                xoff = LL::HALO + 4 * (pos[e] + ql);
                xbuf = FA;
                xcomp = 1;
            }
            const int qd = q - nlap - div_before;  // divergence fluxes of faces t0 + 4 qd .. + 3
            if (qd >= 0 && qd < nd) {
                xsrc = SF + fdiv_ix(n, nr, p, e, k0, t0 + 4 * qd);
                xstep = (n + 3) & ~3;
                xoff = LL::HALO + 4 * NF + pos[e] + 4 * qd;
                xbuf = FA;
                xcomp = 1;
            }
            lap_before += cnt[e];
            div_before += nd;
        }
    }
    // Layer pipeline.  Layers k0 .. kend-1 go through LDS (kend includes the
    // layer above the chunk, the radial neighbour of its last layer).  Two
    // register sets hold the layers in flight: the set of iteration k holds
    // layer k+2, goes to LDS at the start of the iteration and is reloaded
    // with layer k+4 at its end.  The loop is unrolled by two so that the sets
    // alternate without register copies (copying a register that a load is
    // still writing waits for that load); an odd chunk runs one more
    // iteration whose output is discarded, so the loop has a single exit.
    const int kend = min(k1 + 1, nr);
    struct Lay {
        V4<T> o, r;  // own cell, extra record
    };
    auto fetch = [&](Lay &L, bool real) {
        L.o = ld4(real ? own_src : zp);
        L.r = ld4(real ? xsrc : zp);
        own_src += own_step;
        xsrc += xstep;
    };
    auto put = [&](int b, const Lay &L) {
#pragma unroll
        for (int c = 0; c < 4; ++c) lds[b * 4 * HC + c * HC + own_h] = L.o.c[c];
#pragma unroll
        for (int c = 0; c < 4; ++c) lds[xoff + b * xbuf + c * xcomp] = L.r.c[c];
    };
    const T *xcol = x + 4 * cell_ix(n, nr, p, ic, jc, 0);
    T *ycol = y + 4 * cell_ix(n, nr, p, ic, jc, k0);
    T *sink = reinterpret_cast<T *>(g.sink) + 4 * threadIdx.x;

    // prologue: every load first (layers k0 .. k0+3, the layer below, the
    // per-layer factors), then the LDS writes
    constexpr int NLF = (kMaxChunk * 8 + NT - 1) / NT;
    const int nlf = (k1 - k0) * 8;
    Lay A0, A1, S0, S1;
    fetch(A0, true);
    fetch(A1, k0 + 1 < kend);
    fetch(S0, k0 + 2 < kend);
    fetch(S1, k0 + 3 < kend);
    const V4<T> xm_raw = ld4(k0 > 0 ? xcol + 4 * (k0 - 1) * kstride : zp);
    T lf[NLF];
#pragma unroll
    for (int q = 0; q < NLF; ++q) lf[q] = T(g.lay[8 * k0 + min(int(threadIdx.x) + q * NT, nlf - 1)]);
    put(0, A0);
    put(1, A1);
#pragma unroll
    for (int q = 0; q < NLF; ++q) {
        const int t = threadIdx.x + q * NT;
        if (t < nlf) layf[t >> 3][t & 7] = lf[q];
    }
    lds_barrier();
    V4<T> xc, xm;
    for (int c = 0; c < 4; ++c) xc.c[c] = lds[c * HC + own_h];
    xm = k0 > 0 ? xm_raw : wall_ghost(xc, rc.kind, m.nv, T(g.wq2_bot));
    // this column's panel-edge faces (edge tiles): xi edge A, eta edge B
    const int fA = sE ? TY + ty : ty, fB = sN ? 2 * TY + TX + tx : 2 * TY + tx;

    auto step = [&](int k, Lay &S) {
        const int b = (k - k0) % 3;
        put((b + 2) % 3, S);  // layer k+2 (past kend: unused) into the buffer of layer k-1, free since the last barrier
        const T *hb = lds + b * 4 * HC;
        const int b1 = (b + 1) % 3;
        V4<T> xp;
        for (int c = 0; c < 4; ++c) xp.c[c] = lds[b1 * 4 * HC + c * HC + own_h];
        if (k + 1 == nr) xp = wall_ghost(xc, rc.kind, m.nv, T(g.wq2_top));
        const T *fb = lds + LL::HALO + b * FA;
        const T *L = layf[k - k0];
        const T irk2 = L[1], rm2 = L[2], rp2 = L[3], irad = L[4], hrad = L[5], ir = L[6];
        auto V = [&](int c, int di, int dj) -> T { return hb[c * HC + own_h + dj * HX + di]; };
        const T inv_lat = irk2 * m.isc;
        V4<T> out;
        T lap[4];
        for (int c = 0; c < 4; ++c) {
            const T v00 = xc.c[c];
            // cross differences shared by the two faces they serve
            const T dy0 = V(c, 0, 1) - V(c, 0, -1), dyE = V(c, 1, 1) - V(c, 1, -1), dyW = V(c, -1, 1) - V(c, -1, -1);
            const T dx0 = V(c, 1, 0) - V(c, -1, 0), dxN = V(c, 1, 1) - V(c, -1, 1), dxS = V(c, 1, -1) - V(c, -1, -1);
            T oE = m.a11E * (V(c, 1, 0) - v00) + m.a12E * (dy0 + dyE);
            T oW = m.a11W * (V(c, -1, 0) - v00) - m.a12W * (dyW + dy0);
            T oN = m.a22N * (V(c, 0, 1) - v00) + m.a12N * (dx0 + dxN);
            T oS = m.a22S * (V(c, 0, -1) - v00) - m.a12S * (dxS + dx0);
            if (EDGE) {  // conservative averaged fluxes on panel-edge faces (selects)
                const T la = fb[4 * fA + c], lb = fb[4 * fB + c];
                oE = sE ? la : oE;
                oW = sW ? la : oW;
                oN = sN ? lb : oN;
                oS = sS ? lb : oS;
            }
            lap[c] = (oE + oW + oN + oS) * inv_lat + (rp2 * (xp.c[c] - v00) - rm2 * (v00 - xm.c[c])) * irad;
        }
        T dE = 0, dW = 0, dN = 0, dS = 0, rad = 0;
        for (int d = 0; d < 3; ++d) {
            const T v00 = xc.c[d];
            dE += m.tE[d] * (v00 + V(d, 1, 0));
            dW += m.tW[d] * (V(d, -1, 0) + v00);
            dN += m.tN[d] * (v00 + V(d, 0, 1));
            dS += m.tS[d] * (V(d, 0, -1) + v00);
            rad += m.nv[d] * (rp2 * (v00 + xp.c[d]) - rm2 * (xm.c[d] + v00));
        }
        dE *= T(0.5); dW *= T(-0.5); dN *= T(0.5); dS *= T(-0.5);
        if (EDGE) {
            const T da = fb[4 * NF + fA], db = fb[4 * NF + fB];
            dE = sE ? da : dE;
            dW = sW ? da : dW;
            dN = sN ? db : dN;
            dS = sS ? db : dS;
        }
        const T div = (dE + dW + dN + dS) * ir * m.isc + rad * hrad;
        out.c[0] = xc.c[0] - clap * lap[0] - ccor * xc.c[1];
        out.c[1] = xc.c[1] - clap * lap[1] + ccor * xc.c[0];
        out.c[2] = xc.c[2] - clap * lap[2];
        out.c[3] = div - cdt * lap[3];
        if constexpr (VT) {  // buoyancy in the velocity rows; the Theta row (no divergence)
            const T th = xc.c[3], b1 = T(rc.c_r1) * L[0] * th;
            const T un = m.nv[0] * xc.c[0] + m.nv[1] * xc.c[1] + m.nv[2] * xc.c[2];
            out.c[0] -= b1 * m.nv[0];
            out.c[1] -= b1 * m.nv[1];
            out.c[2] -= b1 * m.nv[2];
            out.c[3] = th - T(rc.c_th) * lap[3] - T(rc.c_r2) * irk2 * un;
        }
        __builtin_amdgcn_sched_barrier(0);  // layer k+4 into the set just written to LDS
        fetch(S, k + 4 < kend);
        __builtin_amdgcn_sched_barrier(0);
        st4(act && k < k1 ? ycol : sink, out);
        ycol += 4 * kstride;
        xm = xc;
        xc = xp;
        lds_barrier();  // layer k+2 visible; every read of buffer b done
    };
    for (int k = k0; k < k1; k += 2) {
        step(k, S0);
        step(k + 1, S1);
    }
}

}  // namespace csd
