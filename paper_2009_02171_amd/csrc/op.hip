// Matrix-free finite-volume operator y = A x on the cubed-sphere shell
// (Sec. 3.2, eq. divdiscretization; the two systems of Sec. 3.1).
//
// Three kernels per apply:
//   k_ghost     ghost values one cell beyond every panel edge: cubic
//               interpolation along the neighbour panel's first cell layer;
//   k_edgeflux  for every panel-edge face, the mean of the two panels'
//               one-sided outward fluxes (Laplacian of the 4 components and
//               the divergence flux), which makes the scheme conservative;
//   k_op_main   the 11-point stencil: each workgroup owns a TX x TY column
//               tile of one panel and marches over a chunk of k; plane k
//               (with a one-cell halo) is staged in LDS, planes k-1 and k+1
//               of the own column live in registers, and the r-independent
//               metric of the column is loaded once before the march.
#include <algorithm>

#include "op_dev.h"
#include "profile.h"

namespace csd {

template <class T>
__global__ void k_ghost(DevGeom g, const T *__restrict__ x, T *__restrict__ G) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < g.n) ghost_at(g, x, G, int(blockIdx.z), int(blockIdx.y), t);
}

template <class T>
__global__ void k_edgeflux(DevGeom g, const T *__restrict__ x, const T *__restrict__ G, T *__restrict__ SF) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < g.n) edgeflux_at(g, x, G, SF, int(blockIdx.z), int(blockIdx.y), t);
}

// At least two wavefronts per SIMD (FP64: 256 registers, the whole layer
// pipeline in registers without spilling).
template <class T, int TX, int TY, bool VT>
__global__ __launch_bounds__(TX *TY, 2) void k_op_main(DevGeom g, RowCoef rc, int kchunk, int nkc,
                                                    const T *__restrict__ x, const T *__restrict__ G,
                                                    const T *__restrict__ SF, T *__restrict__ y) {
    __shared__ T lds[OpLds<TX, TY>::SIZE];
    __shared__ T layf[kMaxChunk + 1][8];
    const int n = g.n, nr = g.nr;
    const int tilesx = (n + TX - 1) / TX, tiles = tilesx * ((n + TY - 1) / TY);
    // XCD-aware order: workgroups are dealt round-robin over the 8 XCDs; each
    // XCD takes a contiguous range of (panel, chunk, tile), so neighbouring
    // tiles, which share halo cells, meet in the same L2
    const int nblk = gridDim.x, xcd = blockIdx.x % 8, per = nblk / 8, rem = nblk % 8;
    const int lid = xcd * per + min(xcd, rem) + blockIdx.x / 8;
    const int tile = lid % tiles, slab = lid / tiles;
    const int bx = tile % tilesx, by = tile / tilesx;
    const int p = slab / nkc, kc = slab % nkc;
    const int k0 = kc * kchunk, k1 = min(nr, k0 + kchunk);
    const bool edge_tile = bx == 0 || by == 0 || (bx + 1) * TX >= n || (by + 1) * TY >= n;
    if (edge_tile) op_march<T, TX, TY, true, VT>(g, rc, p, bx, by, k0, k1, x, G, SF, y, lds, layf);
    else op_march<T, TX, TY, false, VT>(g, rc, p, bx, by, k0, k1, x, G, SF, y, lds, layf);
}

// The FP64 stencil for large shells, with the layers requested straight into
// LDS.  gfx950's global_load_lds_dwordx4 writes each lane's 16 bytes to LDS
// (at the wave's base + 16 * lane) without passing through registers, so the
// layers in flight cost no registers and the depth of the pipeline is set by
// LDS: six buffers, layers k and k+1 being read while k+2 .. k+5 are in
// flight.  The work per cell is the same as in op_march; the tile is 16x16
// (four waves, two workgroups per CU), for panels wider than the tile, where a
// tile touches at most one xi edge and one eta edge.
//
// A buffer holds 16-byte pieces in two halves (components 0-1, then 2-3); in
// each half the 256 own cells of the tile come first (piece t = thread t),
// then 128 pieces of extra records (piece 256 + t for thread t of the first
// two waves): the 68 border-ring cells of the halo (ring order: S row, N row,
// W column, E column) and, in edge tiles, the averaged edge-face records.
// Threads with nothing to fetch request the zero page, so every wave issues
// the same requests every layer and the waits are fixed counts.
using lds_ptr = __attribute__((address_space(3))) void *;

template <int TX, int TY>
struct DmaLds {
    static constexpr int NT = TX * TY, HX = TX + 2, HY = TY + 2, HC = HX * HY, NRING = HC - NT;
    static constexpr int NXW = 2;                // waves that request extra records
    static constexpr int SLOTS = NT + 64 * NXW;  // 16-byte pieces per half
    static constexpr int HALF = 2 * SLOTS;       // doubles per half
    static constexpr int BUF = 2 * HALF;         // doubles per buffer
    static constexpr int NB = 6;                 // buffers
    static_assert(NRING <= 64 * NXW && NB * BUF * 8 + (kMaxChunk + NB) * 64 <= 80 * 1024, "layout");
};

// s_waitcnt operand: vmcnt(vm), lgkmcnt(0), expcnt not waited for
__host__ __device__ constexpr int wait_imm(int vm) { return (vm & 15) | ((vm >> 4) << 14) | (7 << 4); }

template <int TX, int TY, bool EDGE>
__device__ __forceinline__ void op_march_dma(const DevGeom &g, const RowCoef &rc, int p, int bx, int by, int k0, int k1,
                                             const double *__restrict__ x, const double *__restrict__ G,
                                             const double *__restrict__ SF, double *__restrict__ y, double *const *bufs,
                                             double (*layf)[8]) {
    using T = double;
    using LL = DmaLds<TX, TY>;
    constexpr int NT = LL::NT, HX = LL::HX, HY = LL::HY, NRING = LL::NRING, NXW = LL::NXW, HALF = LL::HALF;
    constexpr int NB = LL::NB, D = NB - 1;
    static_assert(NB == 6, "the loop below is unrolled by six");
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

    // the record of halo position (hx, hy) at layer k0 and its stride per layer
    auto source = [&](int hx, int hy, const T *&src, int64_t &step) {
        const int ii = bx * TX + hx - 1, jj = by * TY + hy - 1;
        const bool iin = ii >= 0 && ii < n, jin = jj >= 0 && jj < n;
        src = zp;
        step = 0;
        if (iin && jin) { src = x + 4 * cell_ix(n, nr, p, ii, jj, k0); step = 4 * kstride; }
        else if (jin && (ii == -1 || ii == n)) { src = G + 4 * ghost_ix(n, nr, p, ii < 0 ? 0 : 1, k0, jj); step = 4 * n; }
        else if (iin && (jj == -1 || jj == n)) { src = G + 4 * ghost_ix(n, nr, p, jj < 0 ? 2 : 3, k0, ii); step = 4 * n; }
    };
    // position of halo border cell (hx, hy) in the ring order
    auto ring_index = [&](int hx, int hy) -> int {
        if (hy == 0) return hx;
        if (hy == HY - 1) return HX + hx;
        if (hx == 0) return 2 * HX + hy - 1;
        return 2 * HX + (HY - 2) + hy - 1;
    };
    const int r = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(r >> 6);
    const T *own_src, *xsrc = zp;
    int64_t own_step, xstep = 0;
    source(tx + 1, ty + 1, own_src, own_step);
    if (r < NRING) {
        int rhx, rhy;
        if (r < HX) { rhx = r; rhy = 0; }
        else if (r < 2 * HX) { rhx = r - HX; rhy = HY - 1; }
        else if (r < 2 * HX + HY - 2) { rhx = 0; rhy = 1 + r - 2 * HX; }
        else { rhx = HX - 1; rhy = 1 + r - 2 * HX - (HY - 2); }
        source(rhx, rhy, xsrc, xstep);
    }
    // Edge tiles: after the ring, one request per edge face (its four
    // Laplacian fluxes), then one per four faces (their divergence fluxes),
    // edges in the order W, E, S, N.  A column on a panel edge reads its
    // face's records from pieces slA / sdA (xi edge) and slB / sdB (eta edge),
    // the divergence flux being value cA4 / cB4 of its four-face record.
    int slA = 0, sdA = 0, cA4 = 0, slB = 0, sdB = 0, cB4 = 0;
    if (EDGE) {
        const bool eW = bx == 0, eE = (bx + 1) * TX >= n, eS = by == 0, eN = (by + 1) * TY >= n;
        const int cA = min(TY, n - by * TY), cB = min(TX, n - bx * TX);
        const int cnt[4] = {eW ? cA : 0, eE ? cA : 0, eS ? cB : 0, eN ? cB : 0};
        const int nlap = cnt[0] + cnt[1] + cnt[2] + cnt[3];
        const int q = r - NRING;
        int lap_before[4], div_before[4];
        int lb = 0, db = 0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            lap_before[e] = lb;
            div_before[e] = db;
            const int t0 = e < 2 ? by * TY : bx * TX;
            const int nd = (cnt[e] + 3) / 4;
            const int ql = q - lb, qd = q - nlap - db;
            if (q >= 0 && ql >= 0 && ql < cnt[e]) {
                xsrc = SF + 4 * ghost_ix(n, nr, p, e, k0, t0 + ql);
                xstep = 4 * int64_t(n);
            }
            if (q >= 0 && qd >= 0 && qd < nd) {
                xsrc = SF + fdiv_ix(n, nr, p, e, k0, t0 + 4 * qd);
                xstep = (n + 3) & ~3;
            }
            lb += cnt[e];
            db += nd;
        }
        const int lbA = sE ? lap_before[1] : lap_before[0], dbA = sE ? div_before[1] : div_before[0];
        const int lbB = sN ? lap_before[3] : lap_before[2], dbB = sN ? div_before[3] : div_before[2];
        slA = NT + NRING + lbA + ty;
        sdA = NT + NRING + nlap + dbA + ty / 4;
        cA4 = ty % 4;
        slB = NT + NRING + lbB + tx;
        sdB = NT + NRING + nlap + dbB + tx / 4;
        cB4 = tx % 4;
    }
    // LDS offset (doubles, first half) of the nine stencil positions
    int noff[3][3];
#pragma unroll
    for (int dj = -1; dj <= 1; ++dj)
#pragma unroll
        for (int di = -1; di <= 1; ++di) {
            const int hx = tx + 1 + di, hy = ty + 1 + dj;
            const bool inside = hx >= 1 && hx <= TX && hy >= 1 && hy <= TY;
            const int slot = inside ? (hy - 1) * TX + (hx - 1) : NT + ring_index(hx, hy);
            noff[dj + 1][di + 1] = 2 * slot;
        }
    const int kend = min(k1 + 1, nr);
    // The LDS destinations are passed through an empty asm statement: the
    // compiler then cannot tie a request to its buffer and adds no wait of its
    // own before the LDS reads (its waits for requests tied to a buffer are
    // not exact across the unrolled steps and drain the pipeline).  The reads
    // are ordered after the requests they depend on by the explicit waits, and
    // the memory clobber after each barrier keeps the compiler from moving
    // LDS accesses across it.
    auto dma = [&](const T *src, double *dst) {
        lds_ptr d = (lds_ptr)dst;
        asm volatile("" : "+s"(d));
        __builtin_amdgcn_global_load_lds(src, d, 16, 0, 0);
    };
    auto request = [&](double *base, bool real) {
        const T *os = real ? own_src : zp;
        dma(os, base + 2 * 64 * wave);
        dma(os + 2, base + HALF + 2 * 64 * wave);
        if (wave < NXW) {
            const T *xs = real ? xsrc : zp;
            dma(xs, base + 2 * (NT + 64 * wave));
            dma(xs + 2, base + HALF + 2 * (NT + 64 * wave));
        }
        own_src += own_step;
        xsrc += xstep;
        // keep one running pointer each (no per-step copies of the addresses)
        asm volatile("" : "+v"(own_src), "+v"(xsrc));
    };
    // Before step k reads layers k and k+1, each wave waits for its own
    // requests of those layers, then a barrier makes every wave's visible (and
    // ends every read of the buffer the step refills).  The counter is in
    // order and counts stores too: after the requests of layer k+1 a wave has
    // issued those of layers k+2 .. k0+4 (prologue) and, per step since k0,
    // one layer's requests and two stores; with P requests per layer and
    // M = min(k - k0, 4) that leaves 3P + 2M younger operations.
    auto wait = [&](auto mm) {
        constexpr int M = decltype(mm)::value;
        __builtin_amdgcn_sched_barrier(0);
        if (wave < NXW) __builtin_amdgcn_s_waitcnt(wait_imm((D - 2) * 4 + M * 2));
        else __builtin_amdgcn_s_waitcnt(wait_imm((D - 2) * 2 + M * 2));
        __builtin_amdgcn_s_barrier();
        asm volatile("" ::: "memory");
        __builtin_amdgcn_sched_barrier(0);
    };
    const T *xcol = x + 4 * cell_ix(n, nr, p, ic, jc, 0);
    T *ycol = y + 4 * cell_ix(n, nr, p, ic, jc, k0);
    T *sink = reinterpret_cast<T *>(g.sink) + 4 * threadIdx.x;

    // prologue: the layer below and the layer factors into registers, layers
    // k0 .. k0+4 requested, the factors to LDS, then the first wait
    constexpr int NLF = (kMaxChunk * 8 + NT - 1) / NT;
    const int nlf = (k1 - k0) * 8;
    const V4<T> xm_raw = ld4(k0 > 0 ? xcol + 4 * (k0 - 1) * kstride : zp);
    T lf[NLF];
#pragma unroll
    for (int q = 0; q < NLF; ++q) lf[q] = T(g.lay[8 * k0 + min(int(threadIdx.x) + q * NT, nlf - 1)]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < D; ++q) request(bufs[q], k0 + q < kend);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int q = 0; q < NLF; ++q) {
        const int t = threadIdx.x + q * NT;
        if (t < nlf) layf[t >> 3][t & 7] = lf[q];
    }
    wait(std::integral_constant<int, 0>());
    auto own4 = [&](const double *hb) -> V4<T> {
        V4<T> v;
        const int o = noff[1][1];
        v.c[0] = hb[o]; v.c[1] = hb[o + 1]; v.c[2] = hb[HALF + o]; v.c[3] = hb[HALF + o + 1];
        return v;
    };
    V4<T> xc = own4(bufs[0]), xm;
    xm = k0 > 0 ? xm_raw : wall_ghost(xc, rc.kind, m.nv, T(g.wq2_bot));

    // The loop is unrolled by NB so that every buffer is a fixed LDS variable
    // in each step: the compiler then sees that a step's LDS reads do not
    // alias the requests in flight into the other buffers and adds no wait of
    // its own.  Steps past the chunk (last chunk only) store to the sink.
    auto step = [&](auto uc, int k, bool first) {
        constexpr int U = decltype(uc)::value;
        constexpr int B = U, B1 = (U + 1) % NB, BQ = (U + D) % NB;
        using std::integral_constant;
        if (U == 0) {
            if (!first) wait(integral_constant<int, D - 1>());
        } else if (U >= D - 1) {
            wait(integral_constant<int, D - 1>());
        } else {
            if (first) wait(integral_constant<int, (U < D - 1 ? U : D - 1)>());
            else wait(integral_constant<int, D - 1>());
        }
        request(bufs[BQ], k + D < kend);
        __builtin_amdgcn_sched_barrier(0);
        const double *hb = bufs[B];
        V4<T> xp = own4(bufs[B1]);
        {
            const bool top = k + 1 == nr;
            const V4<T> wg = wall_ghost(xc, rc.kind, m.nv, T(g.wq2_top));
#pragma unroll
            for (int c = 0; c < 4; ++c) xp.c[c] = top ? wg.c[c] : xp.c[c];
        }
        const T *L = layf[k - k0];  // rows past the chunk exist (unused values)
        const T irk2 = L[1], rm2 = L[2], rp2 = L[3], irad = L[4], hrad = L[5], ir = L[6];
        auto V = [&](int c, int di, int dj) -> T { return hb[noff[dj + 1][di + 1] + (c >> 1) * HALF + (c & 1)]; };
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
            if (EDGE) {
                const T la = hb[2 * slA + (c >> 1) * HALF + (c & 1)], lb = hb[2 * slB + (c >> 1) * HALF + (c & 1)];
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
            const T da = hb[2 * sdA + (cA4 >> 1) * HALF + (cA4 & 1)], db = hb[2 * sdB + (cB4 >> 1) * HALF + (cB4 & 1)];
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
        __builtin_amdgcn_sched_barrier(0);
        st4(act && k < k1 ? ycol : sink, out);
        __builtin_amdgcn_sched_barrier(0);
        ycol += 4 * kstride;
        xm = xc;
        xc = xp;
    };
    for (int k = k0; k < k1; k += NB) {
        const bool first = k == k0;
        step(std::integral_constant<int, 0>(), k, first);
        step(std::integral_constant<int, 1>(), k + 1, first);
        step(std::integral_constant<int, 2>(), k + 2, first);
        step(std::integral_constant<int, 3>(), k + 3, first);
        step(std::integral_constant<int, 4>(), k + 4, first);
        step(std::integral_constant<int, 5>(), k + 5, first);
    }
    __builtin_amdgcn_s_waitcnt(wait_imm(0));  // no request may land after the workgroup ends
}

template <int TX, int TY>
__global__ __launch_bounds__(TX *TY, 2) void k_op_dma(DevGeom g, RowCoef rc, int kchunk, int nkc,
                                                   const double *__restrict__ x, const double *__restrict__ G,
                                                   const double *__restrict__ SF, double *__restrict__ y) {
    constexpr int BUF = DmaLds<TX, TY>::BUF;
    // one LDS variable per buffer (each step names its buffers statically);
    // layer-factor rows past the chunk are read by the discarded steps
    __shared__ __align__(16) double B0[BUF], B1[BUF], B2[BUF], B3[BUF], B4[BUF], B5[BUF];
    __shared__ double layf[kMaxChunk + 6][8];
    double *const bufs[6] = {B0, B1, B2, B3, B4, B5};
    const int n = g.n, nr = g.nr;
    const int tilesx = (n + TX - 1) / TX, tiles = tilesx * ((n + TY - 1) / TY);
    const int nblk = gridDim.x, xcd = blockIdx.x % 8, per = nblk / 8, rem = nblk % 8;
    const int lid = xcd * per + min(xcd, rem) + blockIdx.x / 8;
    const int tile = lid % tiles, slab = lid / tiles;
    const int bx = tile % tilesx, by = tile / tilesx;
    const int p = slab / nkc, kc = slab % nkc;
    const int k0 = kc * kchunk, k1 = min(nr, k0 + kchunk);
    const bool edge_tile = bx == 0 || by == 0 || (bx + 1) * TX >= n || (by + 1) * TY >= n;
    if (edge_tile) op_march_dma<TX, TY, true>(g, rc, p, bx, by, k0, k1, x, G, SF, y, bufs, layf);
    else op_march_dma<TX, TY, false>(g, rc, p, bx, by, k0, k1, x, G, SF, y, bufs, layf);
}

template <class T>
static int32_t launch_all(const csdyn_opctx *ctx, const T *x, T *y, T *G, T *SF, hipStream_t s) {
    const DevGeom &g = ctx->dg;
    const int n = g.n, nr = g.nr;
    RowCoef rc;
    rc.kind = ctx->op.kind;
    rc.dt = ctx->op.dt;
    const bool vt = ctx->op.kind == CSDYN_VT;
    rc.c_lap = ctx->op.kind == CSDYN_BP ? ctx->op.dt * ctx->op.ekman / ctx->op.pm : ctx->op.dt * ctx->op.ekman;
    rc.c_cor = ctx->op.kind == CSDYN_BP ? 0.0 : 2.0 * ctx->op.dt;
    rc.c_th = vt ? ctx->op.dt * ctx->op.ekman / ctx->op.pr : 0.0;
    rc.c_r1 = vt ? ctx->op.dt * ctx->op.ra / ctx->g.ro : 0.0;
    rc.c_r2 = vt ? ctx->op.dt * ctx->op.ekman * ctx->g.ri * ctx->g.ro : 0.0;
    const dim3 eb(64), eg((n + 63) / 64, nr, 24);
    {
        // ghost: 4 neighbour cells read, 1 written; edge flux: 12 cells read, 5 values written
        const double eb_bytes = 24.0 * n * nr * sizeof(T) * (4 * 4 + 4 + 12 * 4 + 5);
        ProfScope ps(sizeof(T) == 8 ? "op_edges" : "op_edges_f32", 6 * int64_t(n) * n * nr, eb_bytes, s);
        hipLaunchKernelGGL(k_ghost<T>, eg, eb, 0, s, g, x, G);
        hipLaunchKernelGGL(k_edgeflux<T>, eg, eb, 0, s, g, x, (const T *)G, SF);
    }
    ProfScope ps(sizeof(T) == 8 ? "op_main" : "op_main_f32", 6 * int64_t(n) * n * nr,
                 6.0 * n * n * nr * 8 * sizeof(T), s);  // x read once, y written once
    // default: the LDS-request kernel for FP64 shells of at least 6 x 96^3
    // cells (measured faster there; at N = 64 and 80 the register kernel is
    // faster), else 16x8; tile 6 asks for it (FP64, N > 16; otherwise 16x8)
    const bool big = int64_t(n) * n * nr >= int64_t(96) * 96 * 96;
    // the velocity-temperature rows are in the register kernel only
    int tile = ctx->tile ? ctx->tile : (sizeof(T) == 8 && n > 16 && big ? 6 : 4);
    if (vt && tile == 6) tile = 4;
    int32_t status = CSDYN_OK;
    auto go = [&](auto tx_c, auto ty_c) {
        constexpr int TX = decltype(tx_c)::value, TY = decltype(ty_c)::value;
        const int tiles = ((n + TX - 1) / TX) * ((n + TY - 1) / TY);
        const int target = 1024 * 256 / (TX * TY);  // workgroups over the k-chunks
        int nkc = std::max(1, std::min(nr, (target + 6 * tiles - 1) / (6 * tiles)));
        nkc = std::max(nkc, (nr + kMaxChunk - 1) / kMaxChunk);
        int kchunk = (nr + nkc - 1) / nkc;
        kchunk = std::min(kMaxChunk, kchunk + (kchunk & 1));  // even: no discarded iteration
        nkc = (nr + kchunk - 1) / kchunk;
        // every panel-edge face record of a tile needs a thread outside the border ring
        constexpr int NT = TX * TY, NRING = (TX + 2) * (TY + 2) - NT;
        const int fx = std::min(TX, n), fy = std::min(TY, n);
        const int need = (n <= TX ? 2 : 1) * (fy + (fy + 3) / 4) + (n <= TY ? 2 : 1) * (fx + (fx + 3) / 4);
        if (need > NT - NRING) {
            set_error("operator: tile %dx%d has too few threads for the edge faces of N=%d", TX, TY, n);
            status = CSDYN_EINVAL;
            return;
        }
        if (vt)
            hipLaunchKernelGGL((k_op_main<T, TX, TY, true>), dim3(tiles * 6 * nkc), dim3(TX * TY), 0, s, g, rc, kchunk,
                               nkc, x, (const T *)G, (const T *)SF, y);
        else
            hipLaunchKernelGGL((k_op_main<T, TX, TY, false>), dim3(tiles * 6 * nkc), dim3(TX * TY), 0, s, g, rc, kchunk,
                               nkc, x, (const T *)G, (const T *)SF, y);
    };
    using std::integral_constant;
    if (tile == 6 && sizeof(T) == 8 && n > 16) {
        constexpr int TX = 16, TY = 16;
        const int tiles = ((n + TX - 1) / TX) * ((n + TY - 1) / TY);
        const int target = 1024 * 256 / (TX * TY);  // workgroups over the k-chunks
        int nkc = std::max(1, std::min(nr, (target + 6 * tiles - 1) / (6 * tiles)));
        nkc = std::max(nkc, (nr + 59) / 60);
        int kchunk = (nr + nkc - 1) / nkc;
        kchunk = std::min(60, (kchunk + 5) / 6 * 6);  // whole trips of the six-step loop
        nkc = (nr + kchunk - 1) / kchunk;
        // extra records of a tile: the ring and at most one xi and one eta edge
        static_assert((TX + 2) * (TY + 2) - TX * TY + 2 * (TY + (TY + 3) / 4) <= 64 * DmaLds<TX, TY>::NXW,
                      "extra records");
        hipLaunchKernelGGL((k_op_dma<TX, TY>), dim3(tiles * 6 * nkc), dim3(TX * TY), 0, s, g, rc, kchunk, nkc,
                           reinterpret_cast<const double *>(x), reinterpret_cast<const double *>(G),
                           reinterpret_cast<const double *>(SF), reinterpret_cast<double *>(y));
    } else if (tile == 1) go(integral_constant<int, 32>(), integral_constant<int, 8>());
    else if (tile == 2) go(integral_constant<int, 16>(), integral_constant<int, 16>());
    else if (tile == 3) go(integral_constant<int, 64>(), integral_constant<int, 4>());
    else if (tile == 4 || tile == 6) go(integral_constant<int, 16>(), integral_constant<int, 8>());
    else go(integral_constant<int, 32>(), integral_constant<int, 4>());
    if (status != CSDYN_OK) return status;
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

// Step 3 (Sec. 3.1): out_c = x_c - dt (grad_h P)_c for c < 3, with central
// differences of P (ghosts from the operator's edge buffer, wall ghosts by the
// operator's rules) and the dual basis at the cell centre; out_3 was set by the
// operator (the divergence of the corrected face fluxes).
__global__ void k_project(DevGeom g, int kind, double dt, const double *__restrict__ x, const double *__restrict__ G,
                          double *__restrict__ out) {
    const int n = g.n, nr = g.nr;
    const int64_t ncell = 6 * int64_t(n) * n * nr;
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    const int i = int(c % n), j = int((c / n) % n), k = int((c / (int64_t(n) * n)) % nr);
    const int p = int(c / (int64_t(n) * n * nr));
    const double pc = x[4 * c + 3];
    const double pip = fetch_ext(g, x, G, p, i + 1, j, k).c[3], pim = fetch_ext(g, x, G, p, i - 1, j, k).c[3];
    const double pjp = fetch_ext(g, x, G, p, i, j + 1, k).c[3], pjm = fetch_ext(g, x, G, p, i, j - 1, k).c[3];
    const double wall = kind == CSDYN_VP ? pc : -pc;
    const double pkp = k + 1 < nr ? x[4 * (c + int64_t(n) * n) + 3] : wall;
    const double pkm = k > 0 ? x[4 * (c - int64_t(n) * n) + 3] : wall;
    const double d1 = (pip - pim) * 0.5 / g.hs, d2 = (pjp - pjm) * 0.5 / g.hs, d3 = (pkp - pkm) * 0.5 / g.hr;
    const double ir = 1.0 / g.rk[k];
    const size_t a = ((size_t(p) * n + j) * n + i) * 3;
    for (int d = 0; d < 3; ++d) {
        const double gr = (d1 * g.gc1[a + d] + d2 * g.gc2[a + d]) * ir + d3 * g.nrm[a + d];
        out[4 * c + d] = x[4 * c + d] - dt * gr;
    }
}

int32_t op_launch(const csdyn_opctx *ctx, const double *x, double *y, hipStream_t s) {
    return launch_all<double>(ctx, x, y, ctx->dg.G, ctx->dg.SF, s);
}

int32_t op_launch_f32(const csdyn_opctx *ctx, const float *x, float *y, float *G32, float *SF32, hipStream_t s) {
    return launch_all<float>(ctx, x, y, G32, SF32, s);
}

}  // namespace csd

// ------------------------------------------------------------------ C ABI
using namespace csd;

extern "C" int32_t csdyn_op_workspace_bytes(const csdyn_grid *g, size_t *bytes) {
    clear_error();
    if (!g || !bytes) { set_error("csdyn_op_workspace_bytes: null argument"); return CSDYN_EINVAL; }
    if (g->n < 4 || g->nr < 1) { set_error("csdyn_op_workspace_bytes: need n >= 4, nr >= 1"); return CSDYN_EINVAL; }
    *bytes = devgeom_bytes(g->n, g->nr);
    return CSDYN_OK;
}

extern "C" int32_t csdyn_op_setup(const csdyn_grid *g, const csdyn_op *op, void *ws, size_t ws_bytes, void *stream,
                                  csdyn_opctx **out) {
    clear_error();
    if (!g || !op || !ws || !out) { set_error("csdyn_op_setup: null argument"); return CSDYN_EINVAL; }
    *out = nullptr;
    if (op->kind != CSDYN_VP && op->kind != CSDYN_BP && op->kind != CSDYN_VT) {
        set_error("csdyn_op_setup: kind must be VP, BP or VT"); return CSDYN_EINVAL;
    }
    if (!(op->dt >= 0) || !(op->ekman > 0) || (op->kind == CSDYN_BP && !(op->pm > 0)) ||
        (op->kind == CSDYN_VT && (!(op->pr > 0) || !std::isfinite(op->ra)))) {
        set_error("csdyn_op_setup: need dt >= 0, ekman > 0, pm > 0 (BP), pr > 0 and a finite ra (VT)"); return CSDYN_EINVAL;
    }
    auto *ctx = new csdyn_opctx();
    ctx->g = *g; ctx->op = *op; ctx->ws = ws; ctx->ws_bytes = ws_bytes;
    int32_t rc = ctx->hg.build(*g);
    if (rc == CSDYN_OK && ws_bytes < devgeom_bytes(g->n, g->nr)) {
        set_error("csdyn_op_setup: workspace %zu < %zu bytes", ws_bytes, devgeom_bytes(g->n, g->nr));
        rc = CSDYN_ENOMEM;
    }
    if (rc == CSDYN_OK) rc = devgeom_setup(ctx->hg, ws, &ctx->dg);
    if (rc == CSDYN_OK && stream) {
        if (hipStreamSynchronize((hipStream_t)stream) != hipSuccess) { set_error("csdyn_op_setup: stream sync failed"); rc = CSDYN_EHIP; }
    }
    if (rc != CSDYN_OK) { delete ctx; return rc; }
    *out = ctx;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_operator_apply(const csdyn_opctx *ctx, const double *x, double *y, void *stream) {
    clear_error();
    if (!ctx || !x || !y) { set_error("csdyn_operator_apply: null argument"); return CSDYN_EINVAL; }
    const size_t nb = size_t(24) * ctx->g.n * ctx->g.n * ctx->g.nr * sizeof(double);
    const char *xa = (const char *)x, *ya = (const char *)y;
    if (xa < ya + nb && ya < xa + nb) { set_error("csdyn_operator_apply: x and y alias"); return CSDYN_EINVAL; }
    return op_launch(ctx, x, y, (hipStream_t)stream);
}

extern "C" int32_t csdyn_project(const csdyn_opctx *ctx, const double *x, double *out, void *stream) {
    clear_error();
    if (!ctx || !x || !out) { set_error("csdyn_project: null argument"); return CSDYN_EINVAL; }
    const size_t nb = size_t(24) * ctx->g.n * ctx->g.n * ctx->g.nr * sizeof(double);
    const char *xa = (const char *)x, *oa = (const char *)out;
    if (xa < oa + nb && oa < xa + nb) { set_error("csdyn_project: x and out alias"); return CSDYN_EINVAL; }
    if (ctx->op.kind == CSDYN_VT) { set_error("csdyn_project: Step 3 belongs to the VP and BP systems"); return CSDYN_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    CSD_TRY(op_launch(ctx, x, out, s));  // out_3 = divergence of the corrected fluxes; fills the ghost buffer
    const int64_t ncell = 6 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr;
    hipLaunchKernelGGL(k_project, dim3(unsigned((ncell + 255) / 256)), dim3(256), 0, s, ctx->dg, ctx->op.kind,
                       ctx->op.dt, x, (const double *)ctx->dg.G, out);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

extern "C" int32_t csdyn_op_set_tile(csdyn_opctx *ctx, int32_t tile) {
    clear_error();
    if (!ctx || tile < 0 || tile > 6) { set_error("csdyn_op_set_tile: tile must be 0..6"); return CSDYN_EINVAL; }
    ctx->tile = tile;
    return CSDYN_OK;
}

extern "C" void csdyn_op_destroy(csdyn_opctx *ctx) { delete ctx; }
