// Device code of the RAS subdomain solves (Sec. 3.3, eq. onelevel), shared by
// the preconditioner's kernel (ras.hip) and the persistent batched Arnoldi
// step (batched.hip): the packed sweep layouts and the L sweep / U sweep /
// restricted scatter of one subdomain by one workgroup.
#pragma once

#include "ras_host.h"

namespace csd {

template <class TF>
struct Pair;
template <>
struct Pair<double> {
    using type = double2;
};
template <>
struct Pair<float> {
    using type = float2;
};

// Device view of one SweepPack (ras_host.h gives the layouts).
template <class TF>
struct DevSweep {
    using TF2 = typename Pair<TF>::type;
    const int32_t *lane_io;    // [nslice*64] ring, per row of a slice (slice*64 + row): L, x index; U, y index
                               // of an owned row; else -1
    const int32_t *lane_next;  // [nslice*64] per row of a slice: ring, L, the row's U-sweep record; box vector,
                               // U, the row's slot
    const TF2 *val;            // factor entries, two per lane (packed layout: an odd width's last ones one per lane)
    const uint4 *addr;         // [64 * nslice] addresses of the dependencies (ring slots or positions), eight per lane
    const int4 *meta;          // [nsd][meta bytes / 16] LDS metadata image of each subdomain's sweep
};

template <class TF>
struct DevRas {
    using TF2 = typename Pair<TF>::type;
    const SdInfo *sd;
    DevSweep<TF> L, U;
    const TF *dinv;  // [U slices * 64] 1/u_ii per row of a U slice
    TF *lres;        // [U slices * 64] ring: the L sweep's result per row of a U slice
    TF *ring;   // [nsd][depth * width] when the ring is not in LDS
    const int32_t *gio;  // box vector: x index of each position, per subdomain from SdInfo::g0
    const int32_t *perm; // [nsd] subdomain of each workgroup
    const int2 *own;     // box vector: {position, y index} of the owned rows, per subdomain from SdInfo::own0
    int depth, width;
};

// One item of a sweep: one slice for one lane, i.e. the lane's part (at most
// eight entries) of its row: values in pairs, 16-bit dependency addresses two
// to a register, the row's input value (or {L result, 1/u_ii}) and output
// index, and the slice's wave-uniform description.  Nothing in it depends on
// values computed in the sweep (inputs come from x or the box vector,
// addresses and factors are constant), so each wavefront requests its items
// well ahead of use; the loads stay in flight across the LDS-scoped barriers
// between levels.
template <class TF, class TV = TF>
struct Item {
    using TF2 = typename Pair<TF>::type;
    uint32_t addr[4];
    TF2 val[4];
    TF2 h;
    TV xv;         // ring, L: the row's input x value
    int32_t xnext; // ring, L: x index of the row the lane takes in this group's next request
    int32_t io;    // ring, L: the row's U-sweep record; U: y index or -1
    int32_t row;   // box vector, U: the row's slot in the box vector
    int32_t wl;    // level << 17 | sl_info; -1 past the wavefront's last slice
    int32_t slot;  // ring slot (box vector, L: position) of the slice's first row
};

// A fixed number of loads per item of a sweep whatever the slice (pairs past
// the slice's width re-read its last pair; consume() masks them), so the
// memory counters always hold the later items' loads in the same order and
// the wait for one group of items never waits for the next.  Lanes past the
// slice's rows (nvalid = rows * lanes per row) read lane 0's data instead of
// their own padding, so the cache lines of the padding are never fetched;
// their results are discarded.
// Ring, L sweep (eight loads): the row's input straight from x, at the x index
// fetched with this group's previous request (xi), the row's U-sweep record
// and the x index for the group's next request (at slice g2, sp2 lanes per
// row, nvalid2 valid lanes).  Ring, U sweep (eight): the row's L result (lres,
// written by the L sweep), 1/u_ii (rec) and the y index.  With the box vector
// in LDS (VEC) the L sweep's inputs and results live there (five loads per
// item) and the U sweep reads 1/u_ii and its row's slot instead of a record
// (seven loads); y is written after the U sweep.
template <class TF, class TV, bool UPPER, bool VEC, bool TAILS, class Rec>
__device__ __forceinline__ void fetch_item(const DevSweep<TF> &S, const Rec *rec, const TF *lres, const TV *xg, int32_t xi,
                                           int64_t g64, int64_t a64, int64_t g2_64, int sp2, int nvalid2,
                                           int64_t off, int w, int sp, int nvalid, Item<TF, TV> &X) {
    const int lane = threadIdx.x % 64, ln = lane < nvalid ? lane : 0;
    // the row's record, stored per row of the slice (every lane of a split row reads it)
    const int64_t rpos = g64 + ((ln * ((65536 + sp - 1) / sp)) >> 16);
    if constexpr (UPPER && VEC) {  // the row's slot and 1/u_ii
        X.row = S.lane_next[rpos];
        X.h.y = rec[rpos];
    } else if constexpr (UPPER) {  // the L result, 1/u_ii and the y index of an owned row
        X.h.x = lres[rpos];
        X.h.y = rec[rpos];
        X.io = S.lane_io[rpos];
    } else if constexpr (!VEC) {  // the input, the row's U-sweep record
        X.xv = xg[max(xi, 0)];
        X.io = S.lane_next[rpos];
    }
    const int lastp = w > 0 ? (w - 1) / 2 : 0;
    if constexpr (TAILS) {
        // packed layout: pairs j < w / 2, and for an odd width the lanes' last
        // entries one per lane after them, read as pairs starting at the lane's
        // own (its neighbour's value in .y is never used), so the wave fetches 8
        // bytes per lane for them instead of a padded pair.  The tail starts
        // where pair w / 2 would, so each load has one wave-uniform base and a
        // lane offset of ln or 2 ln values; the two byte offsets are kept in
        // registers of their own so that each load costs one select, not a
        // variable shift.
        using TF2 = typename Pair<TF>::type;
        using TF2u = TF2 __attribute__((aligned(sizeof(TF))));
        const int np = w >> 1;
        const char *vs = reinterpret_cast<const char *>(S.val) + 2 * off * int64_t(sizeof(TF));
        unsigned b1 = unsigned(ln) * unsigned(sizeof(TF)), b2 = unsigned(ln) * unsigned(2 * sizeof(TF));
        asm volatile("" : "+v"(b1), "+v"(b2));
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int jj = min(j, lastp);
            const bool tail = (w & 1) && jj == np;
            X.val[j] = *reinterpret_cast<const TF2u *>(vs + 128 * sizeof(TF) * jj + (tail ? b1 : b2));
        }
    } else {  // padded layout: every lane's entries in pairs, an odd width's last one padded
#pragma unroll
        for (int j = 0; j < 4; ++j) X.val[j] = S.val[off + int64_t(min(j, lastp)) * 64 + ln];
    }
    const uint4 a = S.addr[a64 + ln];
    X.addr[0] = a.x; X.addr[1] = a.y; X.addr[2] = a.z; X.addr[3] = a.w;
    if constexpr (!UPPER && !VEC) {  // the next request's x index
        const int l2 = lane < nvalid2 ? lane : 0;
        X.xnext = S.lane_io[g2_64 + ((l2 * ((65536 + sp2 - 1) / sp2)) >> 16)];
    }
}

// The value of the next lane (lane l gets lane l + 1's; the last lane 0): a
// DPP move across the whole wavefront, no trip through the LDS crossbar.
__device__ __forceinline__ float wave_next(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), 0x130, 0xf, 0xf, false));
}
__device__ __forceinline__ double wave_next(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), 0x130, 0xf, 0xf, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), 0x130, 0xf, 0xf, false);
    return __hiloint2double(hi, lo);
}

template <class TF, class TV>
__device__ __forceinline__ TF consume(const Item<TF, TV> &X, int w, const TF *ring, TF acc) {
    TF tv[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) tv[q] = ring[(X.addr[q / 2] >> (16 * (q % 2))) & 0xffffu];
#pragma unroll
    for (int q = 0; q < 8; ++q) acc -= (q < w ? (q % 2 ? X.val[q / 2].y : X.val[q / 2].x) : TF(0)) * tv[q];
    return acc;
}

// Barrier between levels.  When the computed values are in LDS (ring or box
// vector) only LDS traffic has to be complete, so the fence is LDS-scoped:
// global loads issued before it (later items) stay in flight.  On this GPU
// family a full fence would also wait for every outstanding global load.
template <bool LDS_ONLY>
__device__ __forceinline__ void level_barrier() {
    if constexpr (LDS_ONLY) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
        __builtin_amdgcn_s_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
    } else {
        __syncthreads();
    }
}

// Group size K: two groups of K items (seven loads each) in flight per
// wavefront, within the 63 loads the in-order memory counter tracks and the
// register budget of the workgroup size (512 threads: 128 registers keep two
// workgroups per compute unit; 1024 threads leave 128).
template <class TF, int NT>
struct SweepShape {
    static constexpr int K = (NT <= 512 && sizeof(TF) == 4) ? 3 : 2;
};

// Per-subdomain slice metadata of one sweep, staged in LDS.
struct Meta {
    int32_t *lev;   // [nlev + 1] first slice of each level (relative)
    int32_t *off;   // [nsl] first value pair, relative to the subdomain's first
    int32_t *wl;    // [nsl] level << 17 | sl_info
    int32_t *slot;  // [nsl] ring slot (box vector, L: position) of the first row
};

// One triangular sweep of one subdomain.  Slices are dealt to wavefronts
// round-robin over the whole sweep (slice g to wavefront g mod nwaves), and a
// wavefront works through its slices in order.  Its slices are requested in
// two groups of K: while one group is processed the other is in flight, and
// a group is requested again as soon as it has been processed, so the wait
// for a group never waits for the other.  Barrier b ends level b: a
// wavefront passes it as soon as it has finished its slices of levels <= b,
// so every row of levels <= b is in LDS before any row of level b + 1 reads
// it.  Every wavefront passes all nlev barriers.  The lanes of a split row add
// their partial sums in a fixed order; the row's first lane writes the result
// to its ring slot (box vector: its position) and, in the ring layout's L
// sweep, to its U-sweep record; the U sweep writes the owned rows to y
// (restricted scatter).
// y[own[q].y] = ring[own[q].x - shift] for q0 <= q < q1: the {position, y
// index} pairs of a round all requested before the first store.
template <class TV, class TF, int NT, int SU>
__device__ __forceinline__ void scatter_owned(const int2 *own, int q0, int q1, int shift, const TF *ring, TV *y) {
    for (int a0 = q0; a0 < q1; a0 += NT * SU) {
        int2 o[SU];
#pragma unroll
        for (int u = 0; u < SU; ++u) o[u] = own[min(a0 + int(threadIdx.x) + u * NT, q1 - 1)];
#pragma unroll
        for (int u = 0; u < SU; ++u)
            if (a0 + int(threadIdx.x) + u * NT < q1) y[o[u].y] = TV(ring[o[u].x - shift]);
    }
}

// Folded box vector (HostRas::folded): values that wait in registers for
// their slots, v[u] for slot t + u NT (t the thread, slots below n), written
// after the barrier that ends level lev: the late rows' inputs in the L
// sweep, which swap places with the early rows' final L results (slots below
// n are the early rows' positions), and those in the U sweep.
template <class TF, bool FOLD>
struct Fold {
    TF v[kFoldRegs];
    int lev, n, fold;
    const int2 *own;  // U sweep: the owned late rows, written out before their slots are reused
    int own_late;
};
template <class TF>
struct Fold<TF, false> {};

template <class TV, class TF, bool UPPER, bool LDS, bool VEC, int NT, bool FOLD, bool TAILS, class Rec>
__device__ __forceinline__ void sweep(const DevSweep<TF> &S, const Meta &M, int sl0, int asl0, int64_t off0, int nlev,
                                      int nsl, TF *ring, const Rec *rec, const TV *xg, TF *lres, TV *y,
                                      Fold<TF, FOLD> &fd) {
    using It = Item<TF, TV>;
    constexpr bool XG = !UPPER && !VEC;  // ring L sweep: inputs read from x in the items
    constexpr int K = SweepShape<TF, NT>::K;
    const int lane = threadIdx.x % 64, nw = NT / 64;
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x / 64);
    int passed = 0;
    // the barrier that ends level `passed`; folded, after level fd.lev the
    // slots of the early rows change hands (first read at level fd.lev + 2):
    // in the L sweep each thread swaps the early rows' L results in its slots
    // with the late rows' inputs in its registers; in the U sweep the owned
    // late rows are written to y, then (after a barrier, since any thread may
    // read any slot) the early rows' L results go back to their slots
    auto barrier = [&]() {
        level_barrier<LDS>();
        if constexpr (FOLD) {
            if (passed == fd.lev) {
                if constexpr (UPPER) {
                    scatter_owned<TV, TF, NT, 1>(fd.own, 0, fd.own_late, fd.fold, ring, y);  // within the sweep's registers
                    level_barrier<LDS>();
                }
#pragma unroll
                for (int u = 0; u < kFoldRegs; ++u) {
                    const int a = int(threadIdx.x) + u * NT;
                    if (a < fd.n) {
                        const TF e = ring[a];
                        ring[a] = fd.v[u];
                        if constexpr (!UPPER) fd.v[u] = e;
                    }
                }
            }
        }
    };
    auto pass_to = [&](const It &n) {
        const int lv = n.wl >= 0 ? n.wl >> 17 : nlev;
        for (; passed < lv; ++passed) barrier();
    };
    if (nsl == 0) {
        for (; passed < nlev; ++passed) barrier();
        return;
    }
    int fg = wv;  // next slice to request (past the end: re-reads the last slice)
    // ring L sweep: a slice's lanes per row and valid lanes from its metadata
    auto lanes = [&](int gg, int &sp, int &nvalid) {
        const int wl = __builtin_amdgcn_readfirstlane(M.wl[gg]);
        sp = ((wl >> 4) & 63) + 1;
        nvalid = ((wl >> 10) & 127) * sp;
    };
    auto request = [&](It (&grp)[K]) {
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const int g = fg + k * nw, gg = min(g, nsl - 1);
            const int wl = __builtin_amdgcn_readfirstlane(M.wl[gg]);
            const int offr = __builtin_amdgcn_readfirstlane(M.off[gg]);
            grp[k].wl = g < nsl ? wl : -1;
            grp[k].slot = __builtin_amdgcn_readfirstlane(M.slot[gg]);
            // this group's next request takes slice g + 2 K nw in this place
            const int gg2 = min(g + 2 * K * nw, nsl - 1);
            int sp2 = 1, nvalid2 = 1;
            if constexpr (XG) lanes(gg2, sp2, nvalid2);
            fetch_item<TF, TV, UPPER, VEC, TAILS>(
                S, rec, lres, xg, XG ? grp[k].xnext : 0, int64_t(sl0 + gg) * 64, int64_t(asl0 + gg) * 64,
                int64_t(sl0 + gg2) * 64, sp2, nvalid2, off0 + offr, wl & 15, ((wl >> 4) & 63) + 1,
                ((wl >> 10) & 127) * (((wl >> 4) & 63) + 1), grp[k]);
        }
        fg += K * nw;
        __builtin_amdgcn_sched_barrier(0);
    };
    // process one group; next: the first item of the other group
    auto process = [&](const It (&grp)[K], const It &next) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            const It &it = grp[k];
            if (it.wl < 0) break;
            const int w = it.wl & 15, sp = ((it.wl >> 4) & 63) + 1, nrow = (it.wl >> 10) & 127;
            const int rr = (lane * ((65536 + sp - 1) / sp)) >> 16, first = rr * sp;  // row in the slice
            const bool writer = lane == first && rr < nrow;
            TF v0;  // the row's input, added once (by its first lane)
            if constexpr (XG) v0 = writer ? TF(it.xv) : TF(0);
            else if constexpr (!VEC) v0 = writer ? it.h.x : TF(0);
            else if constexpr (UPPER) v0 = writer ? ring[it.row] : TF(0);
            else v0 = writer ? ring[it.slot + rr] : TF(0);
            TF acc = consume(it, w, ring, v0);
            if (sp > 1) {  // the row's first lane adds its other parts in order (part d arrives after d shifts)
                TF sum = acc, part = acc;
                for (int d = 1; d < sp; ++d) {
                    part = wave_next(part);
                    sum += part;
                }
                acc = sum;
            }
            if constexpr (UPPER) acc *= it.h.y;
            if (writer) {  // box vector: y is written from LDS after the sweep (restricted scatter)
                if constexpr (VEC && UPPER) ring[it.row] = acc;
                else ring[it.slot + rr] = acc;
                if constexpr (UPPER && !VEC) {
                    if (it.io >= 0) y[it.io] = TV(acc);
                } else if constexpr (!VEC) {
                    if (it.io >= 0) lres[it.io] = acc;
                }
            }
            pass_to(k + 1 < K ? grp[k + 1] : next);
        }
        __builtin_amdgcn_sched_barrier(0);
    };
    It A[K], B[K];
    if constexpr (XG) {  // the x indices of the first two requests
#pragma unroll
        for (int k = 0; k < 2 * K; ++k) {
            const int gg = min(wv + k * nw, nsl - 1);
            int sp, nvalid;
            lanes(gg, sp, nvalid);
            const int l = lane < nvalid ? lane : 0;
            const int32_t xi = S.lane_io[int64_t(sl0 + gg) * 64 + ((l * ((65536 + sp - 1) / sp)) >> 16)];
            (k < K ? A[k] : B[k - K]).xnext = xi;
        }
    }
    request(A);
    request(B);
    pass_to(A[0]);
    while (A[0].wl >= 0) {
        process(A, B[0]);
        request(A);
        process(B, A[0]);
        request(B);
    }
    for (; passed < nlev; ++passed) barrier();
    __builtin_amdgcn_s_waitcnt(0);  // requests past the end
}


// Pointers into the LDS copy of one sweep's slice metadata (the layout of
// meta_bytes_for and of the per-subdomain images).
__device__ __forceinline__ void meta_pointers(unsigned char *base, int meta_lev, int meta_sl, Meta &M) {
    M.lev = reinterpret_cast<int32_t *>(base);
    M.off = reinterpret_cast<int32_t *>(base + ((size_t(meta_lev) + 1) * 4 + 15) / 16 * 16);
    M.wl = M.off + meta_sl;
    M.slot = M.wl + meta_sl;
}

// One subdomain per workgroup (item `blk` solves subdomain perm[blk]): L
// sweep, U sweep with restricted scatter.  The ring of the last `depth`
// levels is in LDS when LDS = true, else in the workspace, and the L sweep's
// items read their inputs from x; with VEC (always in LDS) the whole box
// vector is there instead: a gather (coalesced over the L-sweep order) writes
// x into it, the L sweep overwrites it with its results and the U sweep with
// its own.
template <class TV, class TF, bool LDS, bool VEC, int NT, bool FOLD = false, bool TAILS = false>
__device__ __forceinline__ void ras_block(const DevRas<TF> &R, int meta_lev, int meta_sl, const TV *__restrict__ x,
                                          TV *__restrict__ y, int blk, unsigned char *ras_smem) {
    static_assert(LDS || !VEC, "the box vector lives in LDS");
    static_assert(VEC || !FOLD, "only a box vector is folded");
    const int sdi = __builtin_amdgcn_readfirstlane(R.perm[blk]);
    const SdInfo I = R.sd[sdi];
    const int ring_n = R.depth * R.width;
    TF *ring = LDS ? reinterpret_cast<TF *>(ras_smem + meta_bytes_for(meta_sl, meta_lev))
                   : R.ring + int64_t(sdi) * ring_n;
    if constexpr (!VEC)
        for (int a = threadIdx.x; a < ring_n; a += NT) ring[a] = TF(0);
    // slice metadata: the L sweep's image to LDS now, the U sweep's (up to
    // MU 16-byte pieces per thread) requested now and written after the L sweep
    Meta M;
    meta_pointers(ras_smem, meta_lev, meta_sl, M);
    using I4 = int __attribute__((ext_vector_type(4)));
    const int n16 = int(meta_bytes_for(meta_sl, meta_lev) / 16);
    I4 *md = reinterpret_cast<I4 *>(ras_smem);
    {
        const I4 *img = reinterpret_cast<const I4 *>(R.L.meta) + size_t(sdi) * n16;
        for (int a = threadIdx.x; a < n16; a += NT) md[a] = img[a];
    }
    constexpr int MU = 2;
    const I4 *uimg = reinterpret_cast<const I4 *>(R.U.meta) + size_t(sdi) * n16;
    const I4 up0 = uimg[min(int(threadIdx.x), n16 - 1)];
    const I4 up1 = uimg[min(int(threadIdx.x) + NT, n16 - 1)];
    Fold<TF, FOLD> fd;
    if constexpr (VEC) {
        // the box vector in L-sweep order: position a holds x[gio[a]];
        // GU positions per thread per round, all index loads and then all
        // value loads in flight together (one round for boxes of up to
        // GU * NT rows).  Folded: positions from I.fold on wait in registers.
        constexpr int GU = 24;
        const int32_t *gi = R.gio + I.g0;
        int nrows = I.nrows;
        if constexpr (FOLD) {
            fd.lev = I.fold_lev;
            fd.n = nrows - I.fold;
            fd.fold = I.fold;
            fd.own = R.own + I.own0;
            fd.own_late = I.own_late;
            int32_t io[kFoldRegs];
#pragma unroll
            for (int u = 0; u < kFoldRegs; ++u) io[u] = gi[I.fold + min(int(threadIdx.x) + u * NT, fd.n - 1)];
#pragma unroll
            for (int u = 0; u < kFoldRegs; ++u) fd.v[u] = TF(x[io[u]]);
            nrows = I.fold;
        }
        for (int a0 = 0; a0 < nrows; a0 += NT * GU) {
            int32_t io[GU];
            TV v[GU];
#pragma unroll
            for (int u = 0; u < GU; ++u) io[u] = gi[min(a0 + int(threadIdx.x) + u * NT, nrows - 1)];
#pragma unroll
            for (int u = 0; u < GU; ++u) v[u] = x[io[u]];
#pragma unroll
            for (int u = 0; u < GU; ++u) {
                const int a = a0 + int(threadIdx.x) + u * NT;
                if (a < nrows) ring[a] = TF(v[u]);
            }
        }
    }  // ring: the L sweep's items read their inputs from x
    __syncthreads();
    sweep<TV, TF, false, LDS, VEC, NT, FOLD, TAILS>(R.L, M, I.slL0, I.aslL0, I.offL0, I.levL1 - I.levL0, I.nslL, ring,
                                             static_cast<const TF *>(nullptr), x, R.lres, y,
                                             fd);
    __syncthreads();  // L results visible; the U metadata replaces the L metadata
    if constexpr (FOLD) fd.lev = I.fold_levU;  // the early rows' L results (in fd.v) go back after this U level
    if (int(threadIdx.x) < n16) md[threadIdx.x] = up0;
    if (int(threadIdx.x) + NT < n16) md[threadIdx.x + NT] = up1;
    for (int a = threadIdx.x + MU * NT; a < n16; a += NT) md[a] = uimg[a];
    __syncthreads();
    sweep<TV, TF, true, LDS, VEC, NT, FOLD, TAILS>(R.U, M, I.slU0, I.aslU0, I.offU0, I.levU1 - I.levU0, I.nslU, ring, R.dinv,
                                            static_cast<const TV *>(nullptr), R.lres, y, fd);
    if constexpr (VEC) {  // restricted scatter of the owned rows from LDS (folded: all but the late ones, which
                          // were written before their slots were reused, have slot = position)
        const int2 *own = R.own + I.own0;
        scatter_owned<TV, TF, NT, 16>(own, FOLD ? I.own_late : 0, 4 * I.nown, 0, ring, y);
    }
}

// Device view of the fine one-level RAS of a preconditioner with FP32 factors
// (for the persistent batched Arnoldi step): mode 0 keeps the ring of recent
// levels in device memory, 1 keeps it in LDS, 2 keeps the whole box vector in
// LDS; lds_bytes is the dynamic LDS one subdomain needs.  CSDYN_EINVAL unless
// the preconditioner is one-level with FP32 factors.
struct RasView {
    DevRas<float> R;
    int meta_lev = 0, meta_sl = 0, nsd = 0, mode = 0;
    int threads = 256;  // workgroup width of the sweeps: 256, 512 or 1024
    size_t lds_bytes = 0;
    double bytes = 0;  // algorithmic bytes of one apply (FP32 factors once, FP64 gather and owned write)
};
int32_t ras_view_f32(const csdyn_ras *pc, RasView &v);

}  // namespace csd
