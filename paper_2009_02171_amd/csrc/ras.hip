// RAS preconditioner on the GPU (Sec. 3.3): one-level restricted additive
// Schwarz with ILU(0) subdomain solves (eq. onelevel) and the hybrid two-level
// preconditioner (eq. twolevel, coarsesolve, finesolve).
//
// k_ras: one workgroup per subdomain.  It gathers x on the overlapping box
// into a scratch vector, runs the L sweep and then the U sweep level by
// level (a workgroup barrier between levels; the rows of one level are
// independent), and writes only the owned cells (restricted scatter, so the
// writes of different workgroups are disjoint).  A wavefront works on slices
// of 64 lanes (a lane holds at most eight entries of a row; wider rows are
// split over adjacent lanes), reads a lane's entries with 16-byte loads, and
// requests its next slices a group ahead, so that one level's critical path
// is LDS reads, a short FMA chain and a barrier rather than a memory latency.
#include <algorithm>
#include <cstring>
#include <memory>
#include <mutex>
#include <type_traits>

#include "krylov.h"
#include "profile.h"
#include "ras_dev.h"

namespace csd {

template <class TV, class TF, bool LDS, bool VEC, int NT, bool FOLD = false, bool TAILS = false>
__global__ __launch_bounds__(NT) void k_ras(DevRas<TF> R, int meta_lev, int meta_sl, const TV *__restrict__ x,
                                            TV *__restrict__ y) {
    extern __shared__ __align__(16) unsigned char ras_smem[];
    ras_block<TV, TF, LDS, VEC, NT, FOLD, TAILS>(R, meta_lev, meta_sl, x, y, int(blockIdx.x), ras_smem);
}

// restriction: mean of the 8 children; prolongation: copy to the children
template <class T>
__global__ void k_restrict(const T *__restrict__ xf, T *__restrict__ xc, int nc, int nrc) {
    const int64_t ncell = 6 * int64_t(nc) * nc * nrc;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    const int nf = 2 * nc, nrf = 2 * nrc;
    for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < 4 * ncell; q += stride) {
        const int c = int(q % 4);
        int64_t cell = q / 4;
        const int I = int(cell % nc); cell /= nc;
        const int J = int(cell % nc); cell /= nc;
        const int K = int(cell % nrc);
        const int p = int(cell / nrc);
        T s = 0;
        for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di)
                    s += xf[4 * (((int64_t(p) * nrf + 2 * K + dk) * nf + 2 * J + dj) * nf + 2 * I + di) + c];
        xc[q] = s * T(0.125);
    }
}

template <class T>
__global__ void k_prolong(const T *__restrict__ xc, T *__restrict__ xf, int nc, int nrc) {
    const int nf = 2 * nc, nrf = 2 * nrc;
    const int64_t n = 24 * int64_t(nf) * nf * nrf;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t q = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; q < n; q += stride) {
        const int c = int(q % 4);
        int64_t cell = q / 4;
        const int i = int(cell % nf); cell /= nf;
        const int j = int(cell % nf); cell /= nf;
        const int k = int(cell % nrf);
        const int p = int(cell / nrf);
        xf[q] = xc[4 * (((int64_t(p) * nrc + k / 2) * nc + j / 2) * nc + i / 2) + c];
    }
}

static dim3 grid_for(int64_t n) { return dim3(unsigned(std::max<int64_t>(1, std::min<int64_t>(8192, (n + 255) / 256)))); }

// One level of RAS data on the device (factors in TF).
struct OneLevel {
    int nsd = 0;
    int64_t nnz = 0, box_cells = 0, owned_cells = 0;
    int depth = 0, width = 0, meta_lev = 0, meta_sl = 0, max_total_levels = 0;
    bool vec = false;  // box vector in LDS instead of the level ring
    bool folded = false;  // FP64 box vector folded into fold_rows slots
    int box_rows = 0, fold_rows = 0;
    int blocks_per_cu = 0;  // workgroups of the sweep kernel that fit one compute unit
    int threads = 256;
    size_t lds_bytes = 0;
    bool lds_ring = false;
    int precision = 0;
    SdInfo *sd = nullptr;
    int32_t *Lio = nullptr, *Lnext = nullptr, *Uio = nullptr, *Unext = nullptr;
    uint16_t *Laddr = nullptr, *Uaddr = nullptr;
    void *Lval = nullptr, *Uval = nullptr, *lout = nullptr, *ring = nullptr;
    int64_t nU = 0;  // entries per U-sweep row array (U slices * 64)
    // Value layout of the sweep: packed (an odd width's last entries one per
    // lane after the slice's pairs, read unpadded) for FP64 launches with at
    // least one subdomain per compute unit, whose time follows each compute
    // unit's bytes; padded pairs otherwise (FP32, and launches of a few
    // workgroups bound by their chain of levels, where the packed layout's
    // per-load address select costs more than its bytes save).
    bool tails = false;
    int32_t *gio = nullptr, *Lmeta = nullptr, *Umeta = nullptr, *perm = nullptr, *own = nullptr;

    static void layout(Carver &c, const HostRas &H, int precision, int values, OneLevel &o) {
        const size_t fs = precision ? sizeof(float) : sizeof(double);
        o.nsd = H.nsd; o.nnz = H.nnz; o.box_cells = H.box_cells; o.owned_cells = H.owned_cells;
        o.depth = H.ring_depth; o.width = H.ring_width; o.meta_lev = H.max_levels; o.meta_sl = H.max_slices;
        o.max_total_levels = H.max_total_levels; o.precision = precision;
        o.vec = H.box_vector; o.box_rows = H.box_rows;
        if (values == 0) {
            int dev = 0, cus = 0;
            if (hipGetDevice(&dev) == hipSuccess &&
                hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
                o.tails = precision == 0 && H.nsd >= cus;
        } else {
            o.tails = values == 1;  // check_opts allows it for FP64 only
        }
        o.folded = H.folded && precision == 0;
        o.fold_rows = o.folded ? H.fold_rows : 0;
        o.sd = c.take<SdInfo>(H.sd.size());
        // the box vector needs no per-lane indices of the L sweep, no U y indices
        // apart from its pairs and no input records
        const bool ring = !H.box_vector;
        o.Lio = c.take<int32_t>(ring ? H.L.lane_io.size() : 0);
        o.Lnext = c.take<int32_t>(ring ? H.L.lane_next.size() : 0);
        o.Laddr = c.take<uint16_t>(o.folded ? H.fold_Laddr.size() : H.L.addr.size());
        o.Lval = c.take<char>((o.tails ? H.L.val.size() : 2 * size_t(padded_pairs(H.L))) * fs);
        o.Uio = c.take<int32_t>(ring ? H.U.lane_io.size() : 0);
        o.Unext = c.take<int32_t>(H.U.lane_next.size());
        o.Uaddr = c.take<uint16_t>(o.folded ? H.fold_Uaddr.size() : H.U.addr.size());
        o.Uval = c.take<char>((o.tails ? H.U.val.size() : 2 * size_t(padded_pairs(H.U))) * fs);
        o.nU = int64_t(H.U.lane_io.size());
        o.lout = c.take<char>(2 * H.U.lane_io.size() * fs);  // 1/u_ii, then the ring's L results
        o.ring = c.take<char>(size_t(H.nsd) * H.ring_depth * H.ring_width * fs);
        o.gio = c.take<int32_t>(H.gio.size());
        o.Lmeta = c.take<int32_t>(H.L.meta.size());
        o.Umeta = c.take<int32_t>(H.U.meta.size());
        o.perm = c.take<int32_t>(H.perm.size());
        o.own = c.take<int32_t>(H.own.size());
    }

    int32_t upload(const HostRas &H) const {
        auto up = [](void *d, const void *s, size_t b) { return b ? hipMemcpy(d, s, b, hipMemcpyHostToDevice) : hipSuccess; };
        if (folded)  // the late inputs a thread holds (the builder sized the fold for this width)
            for (const SdInfo &I : H.sd)
                if (I.nrows - I.fold > kFoldRegs * threads) {
                    set_error("ras: folded subdomain with %d late rows for %d threads", I.nrows - I.fold, threads);
                    return CSDYN_EINVAL;
                }
        // the padded layout: its own value offsets in the subdomain table and
        // metadata images
        const bool padded = !tails;
        std::vector<int64_t> Loff, Uoff;
        std::vector<SdInfo> psd;
        std::vector<int32_t> pLm, pUm;
        if (padded) {
            Loff = padded_offsets(H.L);
            Uoff = padded_offsets(H.U);
            padded_meta(H, folded ? H.fold_Lmeta : H.L.meta, Loff, Uoff, psd, pLm, pUm);
        }
        const std::vector<SdInfo> &sdv = padded ? psd : H.sd;
        CSD_HIP(up(sd, sdv.data(), sdv.size() * sizeof(SdInfo)));
        const bool ring = !H.box_vector;
        if (ring) {
            CSD_HIP(up(Lio, H.L.lane_io.data(), H.L.lane_io.size() * 4));
            CSD_HIP(up(Lnext, H.L.lane_next.data(), H.L.lane_next.size() * 4));
            CSD_HIP(up(Uio, H.U.lane_io.data(), H.U.lane_io.size() * 4));
        }
        const std::vector<uint16_t> &la = folded ? H.fold_Laddr : H.L.addr, &ua = folded ? H.fold_Uaddr : H.U.addr;
        CSD_HIP(up(Laddr, la.data(), la.size() * 2));
        {  // box vector: the row's slot (folded or not) per U lane
            const std::vector<int32_t> &pos = folded ? H.fold_Upos : H.U.lane_next;
            CSD_HIP(up(Unext, pos.data(), pos.size() * 4));
        }
        CSD_HIP(up(own, H.own.data(), H.own.size() * 4));
        CSD_HIP(up(Uaddr, ua.data(), ua.size() * 2));
        CSD_HIP(up(gio, H.gio.data(), H.gio.size() * 4));
        const std::vector<int32_t> &lm = padded ? pLm : (folded ? H.fold_Lmeta : H.L.meta);
        const std::vector<int32_t> &um = padded ? pUm : H.U.meta;
        CSD_HIP(up(Lmeta, lm.data(), lm.size() * 4));
        CSD_HIP(up(Umeta, um.data(), um.size() * 4));
        CSD_HIP(up(perm, H.perm.data(), H.perm.size() * 4));
        auto upload_as = [&](auto zero) -> int32_t {
            using T = decltype(zero);
            std::vector<T> f;
            for (int pass = 0; pass < 2; ++pass) {
                const SweepPack &P = pass ? H.U : H.L;
                if (padded) {
                    const std::vector<int64_t> &no = pass ? Uoff : Loff;
                    f.resize(2 * size_t(padded_pairs(P)));
                    padded_values(P, no, f.data());
                } else {
                    f.assign(P.val.begin(), P.val.end());
                }
                CSD_HIP(up(pass ? Uval : Lval, f.data(), f.size() * sizeof(T)));
            }
            // 1/u_ii per row of a U slice; the ring's L results follow (written by the L sweep)
            f.assign(H.U.lane_diag.size(), T(0));
            for (size_t a = 0; a < H.U.lane_diag.size(); ++a)
                f[a] = H.U.lane_diag[a] != 0.0 ? T(1.0 / H.U.lane_diag[a]) : T(0);
            CSD_HIP(up(lout, f.data(), f.size() * sizeof(T)));
            return CSDYN_OK;
        };
        return precision ? upload_as(0.0f) : upload_as(0.0);
    }

    template <class TF>
    DevRas<TF> dev() const {
        DevRas<TF> R;
        R.sd = sd;
        using TF2 = typename Pair<TF>::type;
        R.L = DevSweep<TF>{Lio, Lnext, (const TF2 *)Lval, (const uint4 *)Laddr, (const int4 *)Lmeta};
        R.U = DevSweep<TF>{Uio, Unext, (const TF2 *)Uval, (const uint4 *)Uaddr, (const int4 *)Umeta};
        R.dinv = (const TF *)lout;
        R.lres = (TF *)lout + nU;
        R.ring = (TF *)ring;
        R.gio = gio;
        R.perm = perm;
        R.own = reinterpret_cast<const int2 *>(own);
        R.depth = vec ? 1 : depth;
        R.width = vec ? box_rows : width;
        return R;
    }

    template <class TV, class TF, bool LDS, bool VEC, int NT, bool FOLD = false, bool TAILS = false>
    static const void *kernel() { return (const void *)k_ras<TV, TF, LDS, VEC, NT, FOLD, TAILS>; }

    template <class TV, class TF, bool TAILS>
    int32_t set_attr_layout() const {
        const hipFuncAttribute at = hipFuncAttributeMaxDynamicSharedMemorySize;
        const int lb = int(lds_bytes);
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, false, 256, false, TAILS>(), at, lb));
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, false, 512, false, TAILS>(), at, lb));
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, false, 1024, false, TAILS>(), at, lb));
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, false, false, 256, false, TAILS>(), at, lb));
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, false, false, 512, false, TAILS>(), at, lb));
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, false, false, 1024, false, TAILS>(), at, lb));
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, true, 256, false, TAILS>(), at, lb));
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, true, 512, false, TAILS>(), at, lb));
        CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, true, 1024, false, TAILS>(), at, lb));
        if constexpr (sizeof(TF) == 8) {
            CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, true, 256, true, TAILS>(), at, lb));
            CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, true, 512, true, TAILS>(), at, lb));
            CSD_HIP(hipFuncSetAttribute(kernel<TV, TF, true, true, 1024, true, TAILS>(), at, lb));
        }
        return CSDYN_OK;
    }

    template <class TV, class TF>
    int32_t set_attr() const {
        if constexpr (sizeof(TF) == 8) {
            if (tails) return set_attr_layout<TV, TF, true>();
        }
        return set_attr_layout<TV, TF, false>();
    }

    // The ring (or the box vector) goes to LDS when it fits next to the
    // metadata; the workgroup size covers one level's slices with one
    // wavefront each (256..1024).
    int32_t choose_memory() {
        int dev = 0, maxs = 0;
        CSD_HIP(hipGetDevice(&dev));
        CSD_HIP(hipDeviceGetAttribute(&maxs, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        const size_t meta = meta_bytes_for(meta_sl, meta_lev);
        const size_t fs = precision ? sizeof(float) : sizeof(double);
        const size_t rb = vec ? size_t(folded ? fold_rows : box_rows) * fs : size_t(depth) * width * fs;
        if (meta > size_t(maxs)) { set_error("ras: subdomain schedule too large for LDS"); return CSDYN_EINVAL; }
        lds_ring = meta + rb <= size_t(maxs);
        if (vec && !lds_ring) { set_error("ras: subdomain vector does not fit in LDS"); return CSDYN_EINVAL; }
        lds_bytes = meta + (lds_ring ? rb : 0);
        threads = sweep_threads(width);
        if (precision) {
            CSD_TRY((set_attr<double, float>()));
            CSD_TRY((set_attr<float, float>()));
        } else {
            CSD_TRY((set_attr<double, double>()));
        }
        // workgroups per compute unit of the kernel that will run (FP64 inputs)
        auto pick = [&](auto tf) -> const void * {
            using TF = decltype(tf);
            auto nt2 = [&](auto l, auto v, auto f, auto t) -> const void * {
                constexpr bool L = decltype(l)::value, V = decltype(v)::value, F = decltype(f)::value;
                constexpr bool P = decltype(t)::value;
                return threads == 256 ? kernel<double, TF, L, V, 256, F, P>()
                       : threads == 512 ? kernel<double, TF, L, V, 512, F, P>() : kernel<double, TF, L, V, 1024, F, P>();
            };
            auto nt = [&](auto l, auto v, auto f) -> const void * {
                if constexpr (sizeof(TF) == 8) {
                    if (tails) return nt2(l, v, f, std::true_type());
                }
                return nt2(l, v, f, std::false_type());
            };
            using T_ = std::true_type;
            using F_ = std::false_type;
            if (vec && folded) {
                if constexpr (sizeof(TF) == 8) return nt(T_(), T_(), T_());
            }
            if (vec) return nt(T_(), T_(), F_());
            return lds_ring ? nt(T_(), F_(), F_()) : nt(F_(), F_(), F_());
        };
        const void *k = precision ? pick(0.0f) : pick(0.0);
        CSD_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks_per_cu, k, threads, lds_bytes));
        return CSDYN_OK;
    }

    template <class TV, class TF, bool LDS, bool VEC, bool FOLD, bool TAILS>
    void launch_layout(const TV *x, TV *y, hipStream_t s) const {
        const dim3 g(nsd);
        if (threads == 256) hipLaunchKernelGGL((k_ras<TV, TF, LDS, VEC, 256, FOLD, TAILS>), g, dim3(256), lds_bytes, s, dev<TF>(), meta_lev, meta_sl, x, y);
        else if (threads == 512) hipLaunchKernelGGL((k_ras<TV, TF, LDS, VEC, 512, FOLD, TAILS>), g, dim3(512), lds_bytes, s, dev<TF>(), meta_lev, meta_sl, x, y);
        else hipLaunchKernelGGL((k_ras<TV, TF, LDS, VEC, 1024, FOLD, TAILS>), g, dim3(1024), lds_bytes, s, dev<TF>(), meta_lev, meta_sl, x, y);
    }

    template <class TV, class TF, bool LDS, bool VEC, bool FOLD = false>
    void launch_nt(const TV *x, TV *y, hipStream_t s) const {
        if constexpr (sizeof(TF) == 8) {
            if (tails) {
                launch_layout<TV, TF, LDS, VEC, FOLD, true>(x, y, s);
                return;
            }
        }
        launch_layout<TV, TF, LDS, VEC, FOLD, false>(x, y, s);
    }

    template <class TV, class TF>
    void launch(const TV *x, TV *y, hipStream_t s) const {
        if constexpr (sizeof(TF) == 8) {
            if (vec && folded) {
                launch_nt<TV, TF, true, true, true>(x, y, s);
                return;
            }
        }
        if (vec) launch_nt<TV, TF, true, true>(x, y, s);
        else if (lds_ring) launch_nt<TV, TF, true, false>(x, y, s);
        else launch_nt<TV, TF, false, false>(x, y, s);
    }

    template <class TV>
    int32_t apply(const TV *x, TV *y, hipStream_t s) const {
        // factor values once, x gathered on the boxes, y written on the owned cells
        const double bytes = double(nnz) * (precision ? 4 : 8) + double(4 * (box_cells + owned_cells)) * sizeof(TV);
        ProfScope ps(precision ? "ras_f32" : "ras", box_cells, bytes, s);
        if (precision) launch<TV, float>(x, y, s);
        else if constexpr (sizeof(TV) == 8) launch<TV, double>(x, y, s);
        CSD_HIP(hipGetLastError());
        return CSDYN_OK;
    }
};

// Host build result cached between csdyn_ras_workspace_bytes and
// csdyn_ras_setup (same operator and options).
struct HostBuild {
    csdyn_grid g;
    csdyn_op op;
    csdyn_ras_opts o;
    HostRas fine, coarse;  // coarse: levels = 2 only
    HostGeom gc;
    std::shared_ptr<HostBuild> inner;  // levels = 3: the coarse grid's two-level hybrid
};

// The options of the coarse grid's two-level hybrid inside a three-level one:
// half the box size (the same subdomain count), two levels.
static csdyn_ras_opts inner_opts(const csdyn_ras_opts &o) {
    csdyn_ras_opts c = o;
    c.levels = 2;
    for (int a = 0; a < 3; ++a) c.sub[a] = o.sub[a] / 2;
    return c;
}

// One cached host build; the key ignores the precision (the FP64 and FP32
// preconditioners of one operator share the assembly and factorization).
static std::mutex g_cache_mu;
static std::shared_ptr<HostBuild> g_cache;

static bool same_key(const HostBuild &b, const csdyn_grid &g, const csdyn_op &op, const csdyn_ras_opts &o) {
    csdyn_ras_opts a = b.o, c = o;
    a.precision = c.precision = 0;
    a.values = c.values = 0;  // the value layout is chosen at upload
    return std::memcmp(&b.g, &g, sizeof(g)) == 0 && std::memcmp(&b.op, &op, sizeof(op)) == 0 &&
           std::memcmp(&a, &c, sizeof(a)) == 0;
}

static int32_t check_opts(const csdyn_opctx *ctx, const csdyn_ras_opts *o) {
    if (!ctx || !o) { set_error("ras: null argument"); return CSDYN_EINVAL; }
    if (o->levels < 1 || o->levels > 3) { set_error("ras: levels must be 1, 2 or 3"); return CSDYN_EINVAL; }
    if (o->precision != 0 && o->precision != 1) { set_error("ras: precision must be 0 or 1"); return CSDYN_EINVAL; }
    if (o->values < 0 || o->values > 2) { set_error("ras: values must be 0, 1 or 2"); return CSDYN_EINVAL; }
    if (o->values == 1 && o->precision != 0) {
        set_error("ras: the packed value layout (values = 1) is for FP64 factors only");
        return CSDYN_EINVAL;
    }
    if (o->levels == 3 && (ctx->g.n % 4 || ctx->g.nr % 4 || o->sub[0] % 4 || o->sub[1] % 4 || o->sub[2] % 4 ||
                           ctx->g.n / 4 < 4)) {
        set_error("ras: three levels need N, Nr and subdomain sizes divisible by 4, and N/4 >= 4");
        return CSDYN_EINVAL;
    }
    if (o->levels >= 2) {
        if (ctx->g.n % 2 || ctx->g.nr % 2 || o->sub[0] % 2 || o->sub[1] % 2 || o->sub[2] % 2 || ctx->g.n / 2 < 4) {
            set_error("ras: two-level needs even N, Nr and subdomain sizes, and N/2 >= 4");
            return CSDYN_EINVAL;
        }
        if (o->coarse_restart < 1 || o->coarse_restart > kRedStride - 1 || o->coarse_maxit < 1 || !(o->coarse_rtol > 0)) {
            set_error("ras: coarse_restart in [1,32], coarse_maxit >= 1, coarse_rtol > 0");
            return CSDYN_EINVAL;
        }
    }
    return CSDYN_OK;
}

static int32_t host_build(const HostGeom &hg, const csdyn_grid &g, const csdyn_op &op, const csdyn_ras_opts *o,
                          std::shared_ptr<HostBuild> &out) {
    auto b = std::make_shared<HostBuild>();
    b->g = g; b->op = op; b->o = *o;
    CSD_TRY(build_host_ras(hg, op, o->sub, o->overlap, o->storage, b->fine));
    if (o->levels >= 2) {
        csdyn_grid gc = g;
        gc.n /= 2; gc.nr /= 2;
        CSD_TRY(b->gc.build(gc));
        if (o->levels == 2) {
            const int subc[3] = {o->sub[0] / 2, o->sub[1] / 2, o->sub[2] / 2};
            CSD_TRY(build_host_ras(b->gc, op, subc, o->overlap, o->storage, b->coarse));
        } else {
            const csdyn_ras_opts oc = inner_opts(*o);
            CSD_TRY(host_build(b->gc, gc, op, &oc, b->inner));
        }
    }
    out = std::move(b);
    return CSDYN_OK;
}

}  // namespace csd

using namespace csd;

struct csdyn_ras {
    csdyn_ras_opts o;
    const csdyn_opctx *fine_ctx;
    OneLevel fine;
    // two-level
    csdyn_opctx coarse_ctx;
    OneLevel coarse;
    void *cws = nullptr;        // coarse GMRES workspace
    void *buf = nullptr;        // fine/coarse temporaries
    int64_t nf = 0, nc = 0;
    mutable int64_t inner_iters = 0;
    double vol_c = 0;           // total coarse volume
    csdyn_ras_info info{};
    // levels = 3: the coarse grid's two-level hybrid (operator: coarse_ctx), which
    // preconditions the coarse solve; its data lie in this handle's workspace
    std::unique_ptr<csdyn_ras> inner;

    template <class T>
    int32_t two_level(const T *x, T *y, hipStream_t s) const;
};

static void layout_all(Carver &c, const HostBuild &b, const csdyn_ras_opts &o, csdyn_ras &R) {
    OneLevel::layout(c, b.fine, o.precision, o.values, R.fine);
    if (o.levels >= 2) {
        const size_t fs = o.precision ? sizeof(float) : sizeof(double);
        const int64_t nf = 24 * int64_t(b.g.n) * b.g.n * b.g.nr;
        const int64_t nc = 24 * int64_t(b.gc.n) * b.gc.n * b.gc.nr;
        R.nf = nf; R.nc = nc;
        void *cg = c.take<char>(devgeom_bytes(b.gc.n, b.gc.nr));
        R.coarse_ctx.ws = cg;
        if (o.levels == 2) OneLevel::layout(c, b.coarse, o.precision, o.values, R.coarse);
        const bool flex = o.levels == 3;  // the coarse solve's preconditioner holds an inner solve
        const size_t gb = o.precision ? Gmres<float>::bytes(nc, o.coarse_restart, flex)
                                        : Gmres<double>::bytes(nc, o.coarse_restart, flex);
        R.cws = c.take<char>(gb);
        // fine: x32, w, t, y32 ; coarse: rc, ec ; FP32 edge buffers for the fine operator
        R.buf = c.take<char>(4 * nf * fs + 2 * nc * fs + 2 * size_t(24) * b.g.nr * b.g.n * 8 * fs + 1024);
        if (o.levels == 3) {
            R.inner.reset(new csdyn_ras);
            layout_all(c, *b.inner, inner_opts(o), *R.inner);
        }
    }
}

// Upload one level of a laid-out preconditioner (and, for three levels, the
// coarse grid's hybrid into the same workspace) and fill its info.
static int32_t setup_level(csdyn_ras &R, const csdyn_opctx *ctx, const csdyn_ras_opts &o, const HostBuild &b) {
    R.o = o;
    R.fine_ctx = ctx;
    R.info = csdyn_ras_info{};
    auto fill = [](const HostRas &H, int32_t &nsd, int64_t &nnz, int64_t &box, int64_t &own, int64_t &stored, int32_t &lv) {
        nsd = H.nsd; nnz = H.nnz; box = H.box_cells; own = H.owned_cells;
        stored = int64_t(H.L.val.size() + H.U.val.size() + H.U.lane_diag.size()); lv = H.max_total_levels;
    };
    fill(b.fine, R.info.nsd_fine, R.info.nnz_fine, R.info.box_cells_fine, R.info.owned_cells_fine, R.info.stored_fine,
         R.info.max_levels_fine);
    // the coarse grid's one-level RAS: its own (two levels) or the inner hybrid's fine one (three levels)
    const HostRas *hc = o.levels == 2 ? &b.coarse : o.levels == 3 ? &b.inner->fine : nullptr;
    if (hc)
        fill(*hc, R.info.nsd_coarse, R.info.nnz_coarse, R.info.box_cells_coarse, R.info.owned_cells_coarse,
             R.info.stored_coarse, R.info.max_levels_coarse);
    R.info.precision = o.precision;
    CSD_TRY(R.fine.choose_memory());
    CSD_TRY(R.fine.upload(b.fine));
    if (o.levels >= 2) {
        R.coarse_ctx.g = ctx->g;
        R.coarse_ctx.g.n /= 2; R.coarse_ctx.g.nr /= 2;
        R.coarse_ctx.op = ctx->op;
        R.coarse_ctx.hg = b.gc;
        R.coarse_ctx.ws_bytes = devgeom_bytes(b.gc.n, b.gc.nr);
        CSD_TRY(devgeom_setup(R.coarse_ctx.hg, R.coarse_ctx.ws, &R.coarse_ctx.dg));
        if (o.levels == 2) {
            CSD_TRY(R.coarse.choose_memory());
            CSD_TRY(R.coarse.upload(b.coarse));
        }
        double v = 0;
        for (double a : b.gc.vol) v += a;
        R.vol_c = v;
        if (o.levels == 3) CSD_TRY(setup_level(*R.inner, &R.coarse_ctx, inner_opts(o), *b.inner));
    }
    const OneLevel &cl = o.levels == 3 ? R.inner->fine : R.coarse;
    R.info.lds_fine = int32_t(R.fine.lds_bytes);
    R.info.box_in_lds_fine = R.fine.vec ? (R.fine.folded ? 3 : 2) : R.fine.lds_ring;
    R.info.lds_coarse = int32_t(cl.lds_bytes);
    R.info.box_in_lds_coarse = cl.vec ? (cl.folded ? 3 : 2) : cl.lds_ring;
    R.info.blocks_per_cu_fine = R.fine.blocks_per_cu;
    R.info.blocks_per_cu_coarse = o.levels >= 2 ? cl.blocks_per_cu : 0;
    R.info.packed_fine = R.fine.tails;
    R.info.packed_coarse = o.levels >= 2 ? cl.tails : 0;
    R.info.threads_fine = R.fine.threads;
    R.info.threads_coarse = o.levels >= 2 ? cl.threads : 0;
    R.info.structures_fine = b.fine.addr_classes;
    R.info.structures_coarse = hc ? hc->addr_classes : 0;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_ras_workspace_bytes(const csdyn_opctx *ctx, const csdyn_ras_opts *o, size_t *bytes) {
    clear_error();
    if (!bytes) { set_error("ras: null bytes"); return CSDYN_EINVAL; }
    CSD_TRY(check_opts(ctx, o));
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (!g_cache || !same_key(*g_cache, ctx->g, ctx->op, *o)) {
        g_cache.reset();
        CSD_TRY(host_build(ctx->hg, ctx->g, ctx->op, o, g_cache));
    }
    csdyn_ras R;
    Carver c(nullptr);
    layout_all(c, *g_cache, *o, R);
    *bytes = c.off + 256;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_ras_setup(const csdyn_opctx *ctx, const csdyn_ras_opts *o, void *ws, size_t ws_bytes,
                                   void *stream, csdyn_ras **out) {
    clear_error();
    if (!ws || !out) { set_error("ras: null argument"); return CSDYN_EINVAL; }
    *out = nullptr;
    CSD_TRY(check_opts(ctx, o));
    std::shared_ptr<HostBuild> b;
    {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        if (!g_cache || !same_key(*g_cache, ctx->g, ctx->op, *o)) {
            g_cache.reset();
            CSD_TRY(host_build(ctx->hg, ctx->g, ctx->op, o, g_cache));
        }
        b = g_cache;
    }
    auto R = std::make_unique<csdyn_ras>();
    Carver c(ws);
    layout_all(c, *b, *o, *R);
    if (c.off + 256 > ws_bytes) { set_error("ras: workspace %zu < %zu bytes", ws_bytes, c.off + 256); return CSDYN_ENOMEM; }
    CSD_TRY(setup_level(*R, ctx, *o, *b));
    if (stream) CSD_HIP(hipStreamSynchronize((hipStream_t)stream));
    *out = R.release();
    return CSDYN_OK;
}

template <class T>
int32_t csdyn_ras::two_level(const T *x, T *y, hipStream_t s) const {
    const int nc_ = coarse_ctx.g.n, nrc = coarse_ctx.g.nr;
    const int64_t ncell_c = nc / 4;
    T *b0 = (T *)buf;
    T *w = b0 + nf, *t = b0 + 2 * nf;
    T *rc = b0 + 4 * nf, *ec = rc + nc;
    T *G32 = ec + nc, *SF32 = G32 + size_t(24) * fine_ctx->g.nr * fine_ctx->g.n * 4;
    Gmres<T> gm;
    Carver cc(cws);
    gm.carve(cc, nc, o.coarse_restart, inner != nullptr);
    {  // r_c = I_f^c x
        PhaseScope ph(PH_PCI, s);
        {
            ProfScope ps("restrict", nc, double(nf + nc) * sizeof(T), s);
            hipLaunchKernelGGL(k_restrict<T>, grid_for(nc), dim3(256), 0, s, x, rc, nc_, nrc);
            CSD_HIP(hipGetLastError());
        }
        if (fine_ctx->op.kind == CSDYN_VP) {  // coarse Neumann solvability: zero volume-weighted mean of P
            CSD_TRY(Vec<T>::pmoments(rc, coarse_ctx.dg.vol, ncell_c, gm.partial, gm.red, s));
            CSD_TRY(Vec<T>::padd_mean(rc, ncell_c, gm.red, s));  // on the device: no wait for the host
        }
    }
    {  // e_c ~ A_c^{-1} r_c : GMRES(coarse_restart) from 0 to coarse_rtol, coarse one-level RAS
        PhaseScope ph(PH_PCC, s);
        CSD_TRY(Vec<T>::zero(ec, nc, s));
        // a two-level coarse step is a few hundred microseconds of device work, so step j + 1 is
        // enqueued before step j is read back; with three levels a step holds an inner solve that
        // waits for the host itself, and a step past convergence would be a whole wasted solve
        gm.lookahead = inner == nullptr;
        const csdyn_opctx *cctx = &coarse_ctx;
        DevFn<T> Ac;
        if constexpr (sizeof(T) == 8) Ac = [cctx](const T *in, T *outv, hipStream_t st) { return op_launch(cctx, in, outv, st); };
        else Ac = [cctx](const T *in, T *outv, hipStream_t st) { return op_launch_f32(cctx, in, outv, (float *)cctx->dg.G, (float *)cctx->dg.SF, st); };
        const OneLevel *cl = &coarse;
        const csdyn_ras *hy = inner.get();
        DevFn<T> Mc;
        if (hy) Mc = [hy](const T *in, T *outv, hipStream_t st) { return hy->two_level<T>(in, outv, st); };
        else Mc = [cl](const T *in, T *outv, hipStream_t st) { return cl->apply<T>(in, outv, st); };
        GmresResult gr;
        int32_t rcode = gm.solve(Ac, &Mc, rc, ec, o.coarse_maxit, o.coarse_rtol, 0.0, s, gr);
        if (rcode < 0) return rcode;
        inner_iters += gr.iters;
    }
    {  // w = I_c^f e_c ; t = x - A_f w
        PhaseScope ph(PH_PCI, s);
        {
            ProfScope ps("prolong", nf, double(nf + nc) * sizeof(T), s);
            hipLaunchKernelGGL(k_prolong<T>, grid_for(nf), dim3(256), 0, s, ec, w, nc_, nrc);
            CSD_HIP(hipGetLastError());
        }
        if constexpr (sizeof(T) == 8) CSD_TRY(op_launch(fine_ctx, w, t, s));
        else CSD_TRY(op_launch_f32(fine_ctx, w, t, G32, SF32, s));
        CSD_TRY(Vec<T>::axpby(1.0, x, -1.0, t, nf, s));
    }
    {  // y = M_one^{-1} t
        PhaseScope ph(PH_PCF, s);
        CSD_TRY(fine.apply<T>(t, y, s));
    }
    PhaseScope ph(PH_PCI, s);  // y += w
    CSD_TRY(Vec<T>::axpby(1.0, w, 1.0, y, nf, s));
    return CSDYN_OK;
}

namespace csd {
// y = M^{-1} x with FP64 vectors at the boundary.
int32_t ras_apply_d(const csdyn_ras *pc, const double *x, double *y, hipStream_t s) {
    if (pc->o.levels == 1) return pc->fine.apply<double>(x, y, s);
    if (pc->o.precision == 0) return pc->two_level<double>(x, y, s);
    float *b0 = (float *)pc->buf;
    float *x32 = b0, *y32 = b0 + 3 * pc->nf;
    {
        PhaseScope ph(PH_PCI, s);
        CSD_TRY(convert_d2f(x, x32, pc->nf, s));
    }
    CSD_TRY(pc->two_level<float>(x32, y32, s));
    PhaseScope ph(PH_PCI, s);
    return convert_f2d(y32, y, pc->nf, s);
}
int ras_levels(const csdyn_ras *pc) { return pc->o.levels; }
int32_t ras_view_f32(const csdyn_ras *pc, RasView &v) {
    if (pc->o.levels != 1 || pc->o.precision != 1) {
        set_error("ras: a one-level preconditioner with FP32 factors is required here");
        return CSDYN_EINVAL;
    }
    const OneLevel &f = pc->fine;
    v.R = f.dev<float>();
    v.meta_lev = f.meta_lev;
    v.meta_sl = f.meta_sl;
    v.nsd = f.nsd;
    v.mode = f.vec ? 2 : (f.lds_ring ? 1 : 0);
    v.threads = f.threads;
    v.lds_bytes = f.lds_bytes;
    v.bytes = double(f.nnz) * 4 + double(4 * (f.box_cells + f.owned_cells)) * sizeof(double);
    return CSDYN_OK;
}
const csdyn_opctx *ras_fine_ctx(const csdyn_ras *pc) { return pc->fine_ctx; }
int64_t ras_inner_iters(const csdyn_ras *pc, bool reset) {
    const int64_t v = pc->inner_iters;
    if (reset) pc->inner_iters = 0;
    return v;
}
// Iterations of the coarsest solves (three levels), accumulated like ras_inner_iters.
int64_t ras_inner2_iters(const csdyn_ras *pc, bool reset) {
    return pc->inner ? ras_inner_iters(pc->inner.get(), reset) : 0;
}
}  // namespace csd

extern "C" int32_t csdyn_ras_apply(const csdyn_ras *pc, const double *x, double *y, void *stream) {
    clear_error();
    if (!pc || !x || !y) { set_error("ras_apply: null argument"); return CSDYN_EINVAL; }
    const size_t nb = size_t(24) * pc->fine_ctx->g.n * pc->fine_ctx->g.n * pc->fine_ctx->g.nr * sizeof(double);
    const char *xa = (const char *)x, *ya = (const char *)y;
    if (xa < ya + nb && ya < xa + nb) { set_error("ras_apply: x and y alias"); return CSDYN_EINVAL; }
    return ras_apply_d(pc, x, y, (hipStream_t)stream);
}

extern "C" void csdyn_ras_destroy(csdyn_ras *pc) { delete pc; }

extern "C" int32_t csdyn_ras_get_info(const csdyn_ras *pc, csdyn_ras_info *info) {
    clear_error();
    if (!pc || !info) { set_error("ras_get_info: null argument"); return CSDYN_EINVAL; }
    *info = pc->info;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_ras_inspect(const csdyn_grid *g, const csdyn_op *op, const int32_t sub[3], int32_t overlap,
                                     int32_t s, int64_t *nloc, int64_t *nnz, int32_t *gcell, int32_t *owned,
                                     int64_t *rowptr, int32_t *col, double *val) {
    clear_error();
    if (!g || !op || !sub || !nloc || !nnz) { set_error("ras_inspect: null argument"); return CSDYN_EINVAL; }
    HostGeom hg;
    CSD_TRY(hg.build(*g));
    const int sb[3] = {sub[0], sub[1], sub[2]};
    std::vector<int32_t> gc, own, ci;
    std::vector<int64_t> rp;
    std::vector<double> v;
    CSD_TRY(host_subdomain(hg, *op, sb, overlap, s, gc, own, rp, ci, v));
    *nloc = int64_t(gc.size());
    *nnz = int64_t(ci.size());
    if (gcell) {
        std::copy(gc.begin(), gc.end(), gcell);
        std::fill(owned, owned + gc.size(), 0);
        for (int32_t l : own) owned[l] = 1;
    }
    if (rowptr) {
        std::copy(rp.begin(), rp.end(), rowptr);
        std::copy(ci.begin(), ci.end(), col);
        std::copy(v.begin(), v.end(), val);
    }
    return CSDYN_OK;
}

// ------------------------------------------------------------------ GMRES
struct SolveLayout {
    Gmres<double> gm;
    double *bproj;
};

static void solve_layout(Carver &c, const csdyn_opctx *ctx, const csdyn_gmres_opts *o, SolveLayout &L) {
    const int64_t n = 24 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr;
    L.gm.carve(c, n, o->restart, o->flexible != 0);
    L.bproj = c.take<double>(n);
}

extern "C" int32_t csdyn_gmres_workspace_bytes(const csdyn_opctx *ctx, const csdyn_gmres_opts *o, size_t *bytes) {
    clear_error();
    if (!ctx || !o || !bytes) { set_error("gmres: null argument"); return CSDYN_EINVAL; }
    if (o->restart < 1 || o->restart > kRedStride - 1) { set_error("gmres: restart must be in [1, 32]"); return CSDYN_EINVAL; }
    Carver c(nullptr);
    SolveLayout L;
    solve_layout(c, ctx, o, L);
    *bytes = c.off + 256;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_gmres_solve(const csdyn_opctx *ctx, const csdyn_ras *pc, const csdyn_gmres_opts *o,
                                     const double *b, double *x, void *ws, size_t ws_bytes, void *stream,
                                     csdyn_gmres_stats *st) {
    clear_error();
    if (!ctx || !o || !b || !x || !ws) { set_error("gmres: null argument"); return CSDYN_EINVAL; }
    if (o->restart < 1 || o->restart > kRedStride - 1 || o->maxit < 1) { set_error("gmres: restart in [1,32], maxit >= 1"); return CSDYN_EINVAL; }
    if (o->orth != 0 && o->orth != 1) { set_error("gmres: orth must be 0 (CGS) or 1 (CGS2)"); return CSDYN_EINVAL; }
    if (pc && pc->fine_ctx->g.n != ctx->g.n) { set_error("gmres: preconditioner built for another grid"); return CSDYN_EINVAL; }
    if (o->rhs_relative != 0 && o->rhs_relative != 1) { set_error("gmres: rhs_relative must be 0 or 1"); return CSDYN_EINVAL; }
    if (o->timing != 0 && o->timing != 1) { set_error("gmres: timing must be 0 or 1"); return CSDYN_EINVAL; }
    if (o->device_steps < 0 || o->device_steps > 32) { set_error("gmres: device_steps must be in [0, 32]"); return CSDYN_EINVAL; }
    Carver c(ws);
    SolveLayout L;
    solve_layout(c, ctx, o, L);
    if (c.off + 256 > ws_bytes) { set_error("gmres: workspace %zu < %zu bytes", ws_bytes, c.off + 256); return CSDYN_ENOMEM; }
    hipStream_t s = (hipStream_t)stream;
    const int64_t n = L.gm.n, ncell = n / 4;
    L.gm.orth = o->orth;
    L.gm.device_steps = o->device_steps;
    if (o->timing) CSD_TRY(phase_timer_begin(s));
    struct TimerGuard {  // uninstalls the timer on every early return
        ~TimerGuard() { phase_timer_abort(); }
    } timer_guard;
    CSD_TRY(Vec<double>::copy(L.bproj, b, n, s));
    auto project = [&](double *v) -> int32_t {
        CSD_TRY(Vec<double>::pmoments(v, ctx->dg.vol, ncell, L.gm.partial, L.gm.red, s));
        double mom[kRedStride];
        CSD_HIP(hipMemcpyAsync(mom, L.gm.red, sizeof(mom), hipMemcpyDeviceToHost, s));
        CSD_HIP(hipStreamSynchronize(s));
        return Vec<double>::padd(v, ncell, -mom[0] / mom[1], s);
    };
    if (ctx->op.kind == CSDYN_VP) CSD_TRY(project(L.bproj));
    DevFn<double> A = [ctx](const double *in, double *outv, hipStream_t st) { return op_launch(ctx, in, outv, st); };
    DevFn<double> M = [pc](const double *in, double *outv, hipStream_t st) { return ras_apply_d(pc, in, outv, st); };
    if (pc) {
        ras_inner_iters(pc, true);
        ras_inner2_iters(pc, true);
    }
    GmresResult res;
    L.gm.m_phase = pc && ras_levels(pc) == 1 ? PH_PCF : -1;
    int32_t rc = L.gm.solve(A, pc ? &M : nullptr, L.bproj, x, o->maxit, o->rtol, o->atol, s, res, o->rhs_relative != 0);
    if (rc < 0) {
        phase_timer_abort();
        return rc;
    }
    if (ctx->op.kind == CSDYN_VP) CSD_TRY(project(x));
    double t_ms[PH_COUNT + 1] = {0, 0, 0, 0, 0, 0}, span = 0;
    if (o->timing) CSD_TRY(phase_timer_end(s, t_ms, &span));
    CSD_HIP(hipStreamSynchronize(s));
    if (st) {
        std::memset(st, 0, sizeof(*st));
        for (int q = 0; q <= PH_COUNT; ++q) st->t_ms[q] = t_ms[q];
        st->t_span_ms = span;
        st->iters = res.iters;
        st->restarts = res.restarts;
        st->inner_iters = pc ? ras_inner_iters(pc, false) : 0;
        st->inner2_iters = pc ? ras_inner2_iters(pc, false) : 0;
        st->relres_true = res.relres_true;
        st->relres_est = res.relres_est;
        st->res0 = res.res0;
        st->res_true = res.res_true;
        st->bnorm = res.bnorm;
    }
    return rc;
}

// ------------------------------------------------------- residual of a guess
struct ResidualLayout {
    double *r, *t, *partial, *red;
};
static void residual_layout(Carver &c, int64_t n, ResidualLayout &L) {
    L.r = c.take<double>(n);
    L.t = c.take<double>(n);
    L.partial = c.take<double>(kPartialElems);
    L.red = c.take<double>(kRedStride);
}

extern "C" int32_t csdyn_residual_workspace_bytes(const csdyn_opctx *ctx, size_t *bytes) {
    clear_error();
    if (!ctx || !bytes) { set_error("residual: null argument"); return CSDYN_EINVAL; }
    Carver c(nullptr);
    ResidualLayout L;
    residual_layout(c, 24 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr, L);
    *bytes = c.off + 256;
    return CSDYN_OK;
}

// ||b - A x|| with the temporaries of ResidualLayout (shared by the
// workspace entry point and the one without a workspace).
static int32_t residual_norm_with(const csdyn_opctx *ctx, const double *b, const double *x, const ResidualLayout &L,
                                  hipStream_t s, double *norm) {
    const int64_t n = 24 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr, ncell = n / 4;
    CSD_TRY(Vec<double>::copy(L.r, b, n, s));
    double h[kRedStride];
    if (ctx->op.kind == CSDYN_VP) {
        CSD_TRY(Vec<double>::pmoments(L.r, ctx->dg.vol, ncell, L.partial, L.red, s));
        CSD_HIP(hipMemcpyAsync(h, L.red, sizeof(h), hipMemcpyDeviceToHost, s));
        CSD_HIP(hipStreamSynchronize(s));
        CSD_TRY(Vec<double>::padd(L.r, ncell, -h[0] / h[1], s));
    }
    CSD_TRY(op_launch(ctx, x, L.t, s));
    CSD_TRY(Vec<double>::axpby(-1.0, L.t, 1.0, L.r, n, s));
    CSD_TRY(Vec<double>::mdot(L.r, n, 0, L.r, L.partial, L.red, s));
    CSD_HIP(hipMemcpyAsync(h, L.red, sizeof(h), hipMemcpyDeviceToHost, s));
    CSD_HIP(hipStreamSynchronize(s));
    *norm = std::sqrt(h[kRedStride - 1]);
    return CSDYN_OK;
}

extern "C" int32_t csdyn_residual_norm(const csdyn_opctx *ctx, const double *b, const double *x, void *ws,
                                       size_t ws_bytes, void *stream, double *norm) {
    clear_error();
    if (!ctx || !b || !x || !ws || !norm) { set_error("residual: null argument"); return CSDYN_EINVAL; }
    Carver c(ws);
    ResidualLayout L;
    residual_layout(c, 24 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr, L);
    if (c.off + 256 > ws_bytes) { set_error("residual: workspace %zu < %zu bytes", ws_bytes, c.off + 256); return CSDYN_ENOMEM; }
    return residual_norm_with(ctx, b, x, L, (hipStream_t)stream, norm);
}

// ------------------------------------- residual of a guess without a workspace
// The temporaries of residual_norm_with for shells of at most
// CSDYN_NOALLOC_MAX_CELLS cells live in this file-scope device array (one copy
// per GPU, held until the process ends).  In host code its name is not a
// device address: kernels receive the address hipGetSymbolAddress returns for
// the current device.
constexpr int64_t kNoAllocN = 4 * int64_t(CSDYN_NOALLOC_MAX_CELLS);
constexpr size_t kNoAllocBytes = 2 * kNoAllocN * sizeof(double) + (kPartialElems + kRedStride) * sizeof(double) + 4 * 256;
static __device__ __align__(256) char scratch[kNoAllocBytes];

static std::mutex g_scratch_mu;
static void *g_scratch_ptr[64];  // per device: the device address of `scratch`

static int32_t scratch_for_current_device(void **ptr) {
    int dev = 0;
    CSD_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) { set_error("residual_noalloc: device %d out of range", dev); return CSDYN_EINVAL; }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        CSD_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) { set_error("residual_noalloc: no device address for the scratch array"); return CSDYN_EHIP; }
        g_scratch_ptr[dev] = p;
    }
    *ptr = g_scratch_ptr[dev];
    return CSDYN_OK;
}

extern "C" int32_t csdyn_residual_norm_noalloc(const csdyn_opctx *ctx, const double *b, const double *x,
                                               void *stream, double *norm) {
    clear_error();
    if (!ctx || !b || !x || !norm) { set_error("residual_noalloc: null argument"); return CSDYN_EINVAL; }
    const int64_t ncell = 6 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr;
    if (ncell > CSDYN_NOALLOC_MAX_CELLS) {
        set_error("residual_noalloc: %lld cells exceed the maximum of %d (use csdyn_residual_norm)", (long long)ncell,
                  CSDYN_NOALLOC_MAX_CELLS);
        return CSDYN_EINVAL;
    }
    void *base = nullptr;
    CSD_TRY(scratch_for_current_device(&base));
    Carver c(base);
    ResidualLayout L;
    residual_layout(c, 4 * ncell, L);
    if (c.off > kNoAllocBytes) { set_error("residual_noalloc: scratch layout exceeds the array"); return CSDYN_EINVAL; }
    return residual_norm_with(ctx, b, x, L, (hipStream_t)stream, norm);
}
