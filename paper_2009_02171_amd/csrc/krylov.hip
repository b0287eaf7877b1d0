// Vector kernels and the restarted (F)GMRES engine (Sec. 3.3, right
// preconditioning, eq. newlinear and the stopping rule after it).
//
// Orthogonalisation is classical Gram-Schmidt as two bandwidth passes over
// the basis (a multi-dot that reads w and V_0..V_j once, then a multi-update
// that also returns ||w||^2); orth = 1 always adds one re-orthogonalisation
// pass (CGS2, its dot products fused into the first update pass), orth = 0
// never does.  Reductions are wavefront shuffles, then a fixed-order two-stage
// sum over blocks, so results are bitwise reproducible.
#include <algorithm>
#include <cmath>
#include <deque>
#include <utility>

#include "krylov_dev.h"
#include "profile.h"

namespace csd {

template <class T>
__global__ __launch_bounds__(kBlk) void k_mdot(const T *__restrict__ V, int64_t n, int cnt, const T *__restrict__ w,
                                               T *__restrict__ partial) {
    mdot_block(V, n, cnt, w, partial, int(blockIdx.x), int(gridDim.x));
}

template <class T>
__global__ __launch_bounds__(kBlk) void k_mupdate(T *__restrict__ w, const T *__restrict__ V, int64_t n, int cnt,
                                                  const T *__restrict__ h, T *__restrict__ partial) {
    mupdate_block(w, V, n, cnt, h, partial, int(blockIdx.x), int(gridDim.x));
}

template <class T>
__global__ void k_scale(T *w, int64_t n, T a) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) w[i] *= a;
}

// v_{j+1} = w / ||w|| with the norms the reduction left on the device (ww:
// ||w||^2 before the projection, nn: after it), the same arithmetic as the
// host's; on a happy breakdown (||w|| <= 1e-14 of its norm before the
// projection) w is left as it is.  With rb, block 0 first copies the nrb
// reduction values red[] to rb (pinned host memory the host reads for the
// step's Hessenberg column), which saves a copy launch per step.
template <class T>
__global__ void k_scale_arnoldi(T *w, int64_t n, const T *ww, const T *nn, const T *red, int nrb, T *rb) {
    if (rb && blockIdx.x == 0)
        for (int i = threadIdx.x; i < nrb; i += blockDim.x) rb[i] = red[i];
    const double hn = sqrt(fmax(double(*nn), 0.0));
    if (hn <= 1e-14 * sqrt(double(*ww))) return;
    const T a = T(1.0 / hn);
    // 16-byte accesses (every vector length is a multiple of 24)
    using VT = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    VT *wv = reinterpret_cast<VT *>(w);
    const int64_t nv = n / W, stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nv; i += stride) {
        VT v = wv[i];
#pragma unroll
        for (int e = 0; e < W; ++e) Vec16<T>::set(v, e, Vec16<T>::get(v, e) * a);
        wv[i] = v;
    }
}

// The same for one Gram-Schmidt pass, with ||w||^2 after the projection summed
// here from the update pass's nbp block partials (every workgroup sums them
// in the order of k_reduce, so the value is the same), which saves the
// reduction's launch: block 0 stores it at *nn_out and copies the step's
// reductions, that one included, to rb.
template <class T>
__global__ __launch_bounds__(256) void k_scale_arnoldi_sum(T *w, int64_t n, const T *ww, const T *partial, int nbp,
                                                           T *nn_out, const T *red, int nrb, T *rb) {
    __shared__ T sred[kRedStride];
    reduce_block<T, 256>(partial, nbp, 0, sred);
    __syncthreads();
    const T nn = sred[kRedStride - 1];
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) *nn_out = nn;
        for (int i = threadIdx.x; i < nrb; i += blockDim.x) rb[i] = i == nrb - 1 ? nn : red[i];
    }
    const double hn = sqrt(fmax(double(nn), 0.0));
    if (hn <= 1e-14 * sqrt(double(*ww))) return;
    const T a = T(1.0 / hn);
    using VT = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    VT *wv = reinterpret_cast<VT *>(w);
    const int64_t nv = n / W, stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < nv; i += stride) {
        VT v = wv[i];
#pragma unroll
        for (int e = 0; e < W; ++e) Vec16<T>::set(v, e, Vec16<T>::get(v, e) * a);
        wv[i] = v;
    }
}

// Rotation state of a restart cycle: H, cs, sn and the header cleared, g =
// (beta, 0, ...).
__global__ void k_hess_reset(double *gs, int m, double beta) {
    const int total = (m + 1) * m + 3 * m + 1 + 8;
    for (int a = threadIdx.x; a < total; a += blockDim.x) gs[a] = 0.0;
    __syncthreads();
    if (threadIdx.x == 0) gs[(m + 1) * m + 2 * m] = beta;
}

// Arnoldi step j's Hessenberg column from the step's reductions (the same
// arithmetic as the host path): h_ij = V_i . w (plus the re-orthogonalisation
// pass), h_{j+1,j} = ||w||; the previous rotations applied to the column, the
// new rotation chosen to zero h_{j+1,j}, g rotated, the estimate |g_{j+1}|
// compared with tol.  Once the cycle has stopped (converged, happy breakdown
// or a non-finite column) later steps leave the state alone.
template <class T>
__global__ void k_hessenberg(const T *red, int nred, double *gs, int j, int m, double tol) {
    if (threadIdx.x != 0) return;
    double *H = gs, *cs = H + (m + 1) * m, *sn = cs + m, *g = sn + m, *hd = g + m + 1;
    if (hd[1] != 0.0) return;
    for (int i = 0; i <= j; ++i)
        H[i * m + j] = nred == 2 ? double(red[i]) : double(red[i]) + double(red[kRedStride + i]);
    const double ww = double(red[kRedStride - 1]);
    const double nn = double(red[nred * kRedStride - 1]);
    const double hn = sqrt(fmax(nn, 0.0));
    hd[4] = double(j + 1);
    if (!isfinite(hn) || !isfinite(ww)) {
        hd[3] = 1.0;
        hd[1] = 1.0;
        return;
    }
    for (int i = 0; i < j; ++i) {
        const double a = H[i * m + j], c = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * c;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
    }
    const double a = H[j * m + j], c = hn;
    const double den = hypot(a, c);
    cs[j] = a / den;
    sn[j] = c / den;
    H[j * m + j] = den;
    H[(j + 1) * m + j] = 0.0;
    g[j + 1] = -sn[j] * g[j];
    g[j] = cs[j] * g[j];
    const double est = fabs(g[j + 1]);
    hd[0] = est;
    if (est <= tol || hn <= 1e-14 * sqrt(ww)) {
        hd[2] = 1.0;
        hd[1] = 1.0;
    }
}

// 16-byte accesses when both vectors are 16-byte aligned and the length is a
// multiple of the width (every system vector's length is a multiple of 24)
template <class T>
__device__ __forceinline__ bool vec16_ok(const void *a, const void *b, int64_t n) {
    return n % Vec16<T>::W == 0 && ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) & 15) == 0;
}

// y = a x + b y
template <class T>
__global__ void k_axpby(T a, const T *__restrict__ x, T b, T *__restrict__ y, int64_t n) {
    using VT = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    if (vec16_ok<T>(x, y, n)) {
        const VT *xv = reinterpret_cast<const VT *>(x);
        VT *yv = reinterpret_cast<VT *>(y);
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n / W; i += stride) {
            const VT u = xv[i];
            VT v = yv[i];
#pragma unroll
            for (int e = 0; e < W; ++e) Vec16<T>::set(v, e, a * Vec16<T>::get(u, e) + b * Vec16<T>::get(v, e));
            yv[i] = v;
        }
        return;
    }
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = a * x[i] + b * y[i];
}

struct Coefs {
    double c[kMaxRestart];
};

template <class T>
__global__ void k_lincomb(T *__restrict__ x, const T *__restrict__ Z, int64_t n, int cnt, Coefs c) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        T acc = x[i];
        for (int q = 0; q < cnt; ++q) acc += T(c.c[q]) * Z[int64_t(q) * n + i];
        x[i] = acc;
    }
}

template <class T>
__global__ void k_copy(T *__restrict__ d, const T *__restrict__ s, int64_t n) {
    using VT = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    if (vec16_ok<T>(d, s, n)) {
        for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n / W; i += stride)
            reinterpret_cast<VT *>(d)[i] = reinterpret_cast<const VT *>(s)[i];
        return;
    }
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = s[i];
}

template <class T>
__global__ void k_zero(T *d, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) d[i] = T(0);
}

template <class T>
__global__ __launch_bounds__(kBlk) void k_pmoments(const T *__restrict__ x, const double *__restrict__ vol,
                                                   int64_t ncell, T *__restrict__ partial) {
    T acc[kRedStride];
#pragma unroll
    for (int q = 0; q < kRedStride; ++q) acc[q] = 0;
    const int64_t stride = int64_t(gridDim.x) * kBlk;
    for (int64_t c = int64_t(blockIdx.x) * kBlk + threadIdx.x; c < ncell; c += stride) {
        const T v = T(vol[c]);
        acc[0] += v * x[4 * c + 3];
        acc[1] += v;
    }
    block_store(acc, 2, partial, int(blockIdx.x));
}

// x[4 c + 3] -= mom[0] / mom[1] with the moments the reduction left on the
// device (the same double division as the host's, so the same shift)
template <class T>
__global__ void k_padd_mean(T *x, int64_t ncell, const T *mom) {
    const T c = T(-double(mom[0]) / double(mom[1]));
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ncell; i += stride) x[4 * i + 3] += c;
}

template <class T>
__global__ void k_padd(T *x, int64_t ncell, T c) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < ncell; i += stride) x[4 * i + 3] += c;
}

__global__ void k_d2f(const double *x, float *y, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = float(x[i]);
}

__global__ void k_f2d(const float *x, double *y, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) y[i] = double(x[i]);
}

// w -= sum_q h[q] V_q, and in the same pass h2[q] = V_q . w_new (the
// re-orthogonalisation dot products of classical Gram-Schmidt, second pass).
template <class T>
__global__ __launch_bounds__(kBlk) void k_mupdate_dot(T *__restrict__ w, const T *__restrict__ V, int64_t n, int cnt,
                                                      const T *__restrict__ h, T *__restrict__ partial) {
    T hq[kRedStride - 1];
#pragma unroll
    for (int q = 0; q < kRedStride - 1; ++q) hq[q] = q < cnt ? h[q] : T(0);
    T acc[kRedStride];
#pragma unroll
    for (int q = 0; q < kRedStride; ++q) acc[q] = 0;
    const int64_t stride = int64_t(gridDim.x) * kBlk;
    for (int64_t i = int64_t(blockIdx.x) * kBlk + threadIdx.x; i < n; i += stride) {
        T vq[kRedStride - 1];
        T wv = w[i];
#pragma unroll
        for (int q = 0; q < kRedStride - 1; ++q) {
            vq[q] = q < cnt ? V[int64_t(q) * n + i] : T(0);
            wv -= hq[q] * vq[q];
        }
        w[i] = wv;
#pragma unroll
        for (int q = 0; q < kRedStride - 1; ++q) acc[q] += vq[q] * wv;
        acc[kRedStride - 1] += wv * wv;
    }
    block_store(acc, cnt, partial, int(blockIdx.x));
}

template <class T>
__global__ __launch_bounds__(1024) void k_reduce(const T *__restrict__ partial, int nb, int cnt, T *__restrict__ out) {
    reduce_block<T, 1024>(partial, nb, cnt, out);
}

static dim3 ew_grid(int64_t n) {
    return dim3(unsigned(std::max<int64_t>(1, std::min<int64_t>(4096, (n + 255) / 256))));
}

#define CSD_LAUNCHED() CSD_HIP(hipGetLastError())

template <class T>
int32_t Vec<T>::mdot(const T *V, int64_t n, int cnt, const T *w, T *partial, T *out, hipStream_t s) {
    const int nb = nblocks(n);
    ProfScope ps(sizeof(T) == 8 ? "mdot" : "mdot_f32", n, double(cnt + 1) * n * sizeof(T), s);
    hipLaunchKernelGGL(k_mdot<T>, dim3(nb), dim3(kBlk), 0, s, V, n, cnt, w, partial);
    hipLaunchKernelGGL(k_reduce<T>, dim3(1), dim3(1024), 0, s, partial, nb, cnt, out);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::mupdate(T *w, const T *V, int64_t n, int cnt, const T *h, T *partial, T *out, hipStream_t s) {
    const int nb = nblocks(n);
    ProfScope ps(sizeof(T) == 8 ? "mupdate" : "mupdate_f32", n, double(cnt + 2) * n * sizeof(T), s);
    hipLaunchKernelGGL(k_mupdate<T>, dim3(nb), dim3(kBlk), 0, s, w, V, n, cnt, h, partial);
    hipLaunchKernelGGL(k_reduce<T>, dim3(1), dim3(1024), 0, s, partial, nb, 0, out);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::mupdate_blocks(T *w, const T *V, int64_t n, int cnt, const T *h, T *partial, hipStream_t s) {
    const int nb = nblocks(n);
    ProfScope ps(sizeof(T) == 8 ? "mupdate" : "mupdate_f32", n, double(cnt + 2) * n * sizeof(T), s);
    hipLaunchKernelGGL(k_mupdate<T>, dim3(nb), dim3(kBlk), 0, s, w, V, n, cnt, h, partial);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::mupdate_dot(T *w, const T *V, int64_t n, int cnt, const T *h, T *partial, T *out, hipStream_t s) {
    const int nb = nblocks(n);
    ProfScope ps(sizeof(T) == 8 ? "mupdate_dot" : "mupdate_dot_f32", n, double(cnt + 2) * n * sizeof(T), s);
    hipLaunchKernelGGL(k_mupdate_dot<T>, dim3(nb), dim3(kBlk), 0, s, w, V, n, cnt, h, partial);
    hipLaunchKernelGGL(k_reduce<T>, dim3(1), dim3(1024), 0, s, partial, nb, cnt, out);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::scale(T *w, int64_t n, double a, hipStream_t s) {
    hipLaunchKernelGGL(k_scale<T>, ew_grid(n), dim3(256), 0, s, w, n, T(a));
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::axpby(double a, const T *x, double b, T *y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby<T>, ew_grid(n), dim3(256), 0, s, T(a), x, T(b), y, n);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::lincomb(T *x, const T *Z, int64_t n, int cnt, const double *c, hipStream_t s) {
    Coefs cf{};
    for (int q = 0; q < cnt && q < kMaxRestart; ++q) cf.c[q] = c[q];
    ProfScope ps("lincomb", n, double(cnt + 2) * n * sizeof(T), s);
    hipLaunchKernelGGL(k_lincomb<T>, ew_grid(n), dim3(256), 0, s, x, Z, n, cnt, cf);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::copy(T *dst, const T *src, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_copy<T>, ew_grid(n), dim3(256), 0, s, dst, src, n);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::zero(T *x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_zero<T>, ew_grid(n), dim3(256), 0, s, x, n);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::pmoments(const T *x, const double *vol, int64_t ncell, T *partial, T *out, hipStream_t s) {
    const int nb = nblocks(ncell);
    hipLaunchKernelGGL(k_pmoments<T>, dim3(nb), dim3(kBlk), 0, s, x, vol, ncell, partial);
    hipLaunchKernelGGL(k_reduce<T>, dim3(1), dim3(1024), 0, s, partial, nb, 2, out);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::padd_mean(T *x, int64_t ncell, const T *mom, hipStream_t s) {
    hipLaunchKernelGGL(k_padd_mean<T>, ew_grid(ncell), dim3(256), 0, s, x, ncell, mom);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template <class T>
int32_t Vec<T>::padd(T *x, int64_t ncell, double c, hipStream_t s) {
    hipLaunchKernelGGL(k_padd<T>, ew_grid(ncell), dim3(256), 0, s, x, ncell, T(c));
    CSD_LAUNCHED();
    return CSDYN_OK;
}

int32_t convert_d2f(const double *x, float *y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_d2f, ew_grid(n), dim3(256), 0, s, x, y, n);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

int32_t convert_f2d(const float *x, double *y, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_f2d, ew_grid(n), dim3(256), 0, s, x, y, n);
    CSD_LAUNCHED();
    return CSDYN_OK;
}

template struct Vec<double>;
template struct Vec<float>;

// ------------------------------------------------------------------ GMRES
template <class T>
size_t Gmres<T>::bytes(int64_t n, int m, bool flexible) {
    Carver c(nullptr);
    Gmres<T> g;
    g.carve(c, n, m, flexible);
    return c.off + 256;
}

template <class T>
void Gmres<T>::carve(Carver &c, int64_t n_, int m_, bool flexible_) {
    n = n_; m = m_; flexible = flexible_;
    V = c.take<T>(size_t(m + 1) * n);
    if (flexible) Z = c.take<T>(size_t(m) * n);
    z = c.take<T>(n);
    r = c.take<T>(n);
    tmp = c.take<T>(n);
    partial = c.take<T>(kPartialElems);
    red = c.take<T>(3 * kRedStride);
    gs = c.take<double>(gs_elems(m));
}

template <class T>
int32_t Gmres<T>::fetch(int cnt, std::vector<T> &out, hipStream_t s) {
    out.resize(kRedStride);
    CSD_HIP(hipMemcpyAsync(out.data(), red, sizeof(T) * kRedStride, hipMemcpyDeviceToHost, s));
    CSD_HIP(hipStreamSynchronize(s));
    (void)cnt;
    return CSDYN_OK;
}

template <class T>
int32_t Gmres<T>::norm(const T *v, double &out, hipStream_t s) {
    CSD_TRY(Vec<T>::mdot(v, n, 0, v, partial, red, s));
    std::vector<T> h;
    CSD_TRY(fetch(0, h, s));
    out = std::sqrt(double(h[kRedStride - 1]));
    return CSDYN_OK;
}

// Pinned host buffers and events for the Arnoldi read-backs: two per solve
// nesting depth on this thread and device (the two-level preconditioner runs
// a coarse solve inside an iteration of the outer solve), kept until the
// process ends.
constexpr size_t kReadBackElems = 2048;  // doubles: a step's reductions or a cycle's rotation state
struct ReadBack {
    void *buf[2] = {nullptr, nullptr};
    void *dbuf[2] = {nullptr, nullptr};  // the same buffers as the device addresses them
    hipEvent_t ev[2] = {nullptr, nullptr};
};

static int32_t readback_for(int depth, ReadBack *&rb) {
    // (device * 64 + depth, buffers); a deque keeps the entries in place while
    // a nested solve appends its own
    static thread_local std::deque<std::pair<int, ReadBack>> pool;
    int dev = 0;
    CSD_HIP(hipGetDevice(&dev));
    const int key = dev * 64 + depth;
    for (auto &e : pool)
        if (e.first == key) { rb = &e.second; return CSDYN_OK; }
    ReadBack r;
    for (int i = 0; i < 2; ++i) {
        CSD_HIP(hipHostMalloc(&r.buf[i], sizeof(double) * kReadBackElems, hipHostMallocDefault));
        CSD_HIP(hipHostGetDevicePointer(&r.dbuf[i], r.buf[i], 0));
        CSD_HIP(hipEventCreateWithFlags(&r.ev[i], hipEventDisableTiming));
    }
    pool.emplace_back(key, r);
    rb = &pool.back().second;
    return CSDYN_OK;
}

static thread_local int t_solve_depth = 0;

template <class T>
int32_t Gmres<T>::solve(const DevFn<T> &A, const DevFn<T> *M, const T *b, T *x, int maxit, double rtol,
                        double atol, hipStream_t s, GmresResult &res, bool rhs_relative) {
    res = GmresResult();
    if (m < 1 || m > kRedStride - 1 || maxit < 1) {
        set_error("gmres: restart must be in [1, %d] and maxit >= 1", kRedStride - 1);
        return CSDYN_EINVAL;
    }
    if (t_solve_depth >= 64) { set_error("gmres: solves nested too deeply"); return CSDYN_EINVAL; }
    ReadBack *rb = nullptr;
    CSD_TRY(readback_for(t_solve_depth, rb));
    struct Depth {
        Depth() { ++t_solve_depth; }
        ~Depth() { --t_solve_depth; }
    } depth_guard;
    std::vector<double> H(size_t(m + 1) * m, 0.0), cs(m), sn(m), gv(m + 1), yv(m);
    // r = b - A x
    {
        PhaseScope ps(PH_OP, s);
        CSD_TRY(A(x, tmp, s));
    }
    CSD_TRY(Vec<T>::copy(r, b, n, s));
    CSD_TRY(Vec<T>::axpby(-1.0, tmp, 1.0, r, n, s));
    double beta0;
    CSD_TRY(norm(r, beta0, s));
    if (!std::isfinite(beta0)) { set_error("gmres: non-finite initial residual"); return CSDYN_EBREAKDOWN; }
    double bnorm = beta0;
    if (rhs_relative) CSD_TRY(norm(b, bnorm, s));
    const double tol = std::max(atol, rtol * (rhs_relative ? bnorm : beta0));
    const int nred = orth == 0 ? 2 : 3;  // reduction blocks read back per iteration
    // Arnoldi step j on the device: z_j = M v_j, w = A z_j, classical
    // Gram-Schmidt (h = V^T w, then w -= V h with ||w||^2 in the same pass;
    // CGS2 re-orthogonalises once, the second dot fused into the update),
    // read-back of h and the norms, v_{j+1} = w / ||w|| from the device norms.
    auto apply_M = [&](const T *in, T *outv) -> int32_t {
        if (m_phase >= 0) {
            PhaseScope ps(Phase(m_phase), s);
            return (*M)(in, outv, s);
        }
        return (*M)(in, outv, s);
    };
    auto apply_A = [&](const T *in, T *outv) -> int32_t {
        PhaseScope ps(PH_OP, s);
        return A(in, outv, s);
    };
    auto launch_step = [&](int j) -> int32_t {
        T *vj = V + size_t(j) * n, *w = V + size_t(j + 1) * n;
        T *zj = flexible ? Z + size_t(j) * n : z;
        if (M) CSD_TRY(apply_M(vj, zj));
        else CSD_TRY(Vec<T>::copy(zj, vj, n, s));
        CSD_TRY(apply_A(zj, w));
        {
            PhaseScope ps(PH_ORTH, s);
            CSD_TRY(Vec<T>::mdot(V, n, j + 1, w, partial, red, s));
            if (orth == 0) {
                CSD_TRY(Vec<T>::mupdate_blocks(w, V, n, j + 1, red, partial, s));
            } else {
                CSD_TRY(Vec<T>::mupdate_dot(w, V, n, j + 1, red, partial, red + kRedStride, s));
                CSD_TRY(Vec<T>::mupdate(w, V, n, j + 1, red + kRedStride, partial, red + 2 * kRedStride, s));
            }
        }
        {
            PhaseScope ps(PH_ORTH, s);  // v_{j+1}, and the step's reductions to the host's buffer
            T *nn = red + nred * kRedStride - 1;
            if (orth == 0)  // ||w||^2 summed from the update pass's partials by this kernel itself
                hipLaunchKernelGGL(k_scale_arnoldi_sum<T>, dim3(std::min<unsigned>(ew_grid(n).x, kMaxBlocks)), dim3(256),
                                   0, s, w, n, (const T *)(red + kRedStride - 1), (const T *)partial,
                                   Vec<T>::nblocks(n), nn, (const T *)red, nred * kRedStride,
                                   static_cast<T *>(rb->dbuf[j % 2]));
            else
                hipLaunchKernelGGL(k_scale_arnoldi<T>, ew_grid(n), dim3(256), 0, s, w, n, red + kRedStride - 1, nn,
                                   (const T *)red, nred * kRedStride, static_cast<T *>(rb->dbuf[j % 2]));
            CSD_LAUNCHED();
        }
        CSD_HIP(hipEventRecord(rb->ev[j % 2], s));
        return CSDYN_OK;
    };
    // device-resident form of step j: the same kernels without the read-back,
    // then the rotation on the device
    auto launch_step_dev = [&](int j) -> int32_t {
        T *vj = V + size_t(j) * n, *w = V + size_t(j + 1) * n;
        T *zj = flexible ? Z + size_t(j) * n : z;
        if (M) CSD_TRY(apply_M(vj, zj));
        else CSD_TRY(Vec<T>::copy(zj, vj, n, s));
        CSD_TRY(apply_A(zj, w));
        PhaseScope ps(PH_ORTH, s);
        CSD_TRY(Vec<T>::mdot(V, n, j + 1, w, partial, red, s));
        if (orth == 0) {
            CSD_TRY(Vec<T>::mupdate(w, V, n, j + 1, red, partial, red + kRedStride, s));
        } else {
            CSD_TRY(Vec<T>::mupdate_dot(w, V, n, j + 1, red, partial, red + kRedStride, s));
            CSD_TRY(Vec<T>::mupdate(w, V, n, j + 1, red + kRedStride, partial, red + 2 * kRedStride, s));
        }
        hipLaunchKernelGGL(k_hessenberg<T>, dim3(1), dim3(64), 0, s, red, nred, gs, j, m, tol);
        CSD_LAUNCHED();
        hipLaunchKernelGGL(k_scale_arnoldi<T>, ew_grid(n), dim3(256), 0, s, w, n, red + kRedStride - 1,
                           red + nred * kRedStride - 1, (const T *)nullptr, 0, (T *)nullptr);
        CSD_LAUNCHED();
        return CSDYN_OK;
    };
    // One restart cycle of at most `limit` steps with device-resident steps:
    // groups of device_steps steps, each followed by a read-back of the
    // rotation header; group k + 1 is enqueued before the host waits for group
    // k.  On return H (rotated) and gv hold the cycle's state for the steps done.
    auto cycle_dev = [&](int limit, double beta_c, int &jdone, bool &stop, double &est_out) -> int32_t {
        hipLaunchKernelGGL(k_hess_reset, dim3(1), dim3(256), 0, s, gs, m, beta_c);
        CSD_LAUNCHED();
        const int hdr = (m + 1) * m + 3 * m + 1;
        int enq = 0, groups = 0, waited = 0;
        auto enqueue_group = [&]() -> int32_t {
            const int j1 = std::min(limit, enq + device_steps);
            for (int j = enq; j < j1; ++j) CSD_TRY(launch_step_dev(j));
            CSD_HIP(hipMemcpyAsync(rb->buf[groups % 2], gs + hdr, sizeof(double) * 8, hipMemcpyDeviceToHost, s));
            CSD_HIP(hipEventRecord(rb->ev[groups % 2], s));
            enq = j1;
            ++groups;
            return CSDYN_OK;
        };
        CSD_TRY(enqueue_group());
        stop = false;
        for (;;) {
            if (enq < limit) CSD_TRY(enqueue_group());
            CSD_HIP(hipEventSynchronize(rb->ev[waited % 2]));
            const double *hd = static_cast<const double *>(rb->buf[waited % 2]);
            ++waited;
            if (hd[3] != 0.0) { set_error("gmres: non-finite Arnoldi vector"); return CSDYN_EBREAKDOWN; }
            if (hd[1] != 0.0) { stop = true; break; }
            if (waited == groups && enq >= limit) break;
        }
        // the rotation state of the steps done (a later group may still be running)
        double *hb = static_cast<double *>(rb->buf[waited % 2]);
        CSD_HIP(hipMemcpyAsync(hb, gs, sizeof(double) * (hdr + 8), hipMemcpyDeviceToHost, s));
        CSD_HIP(hipStreamSynchronize(s));
        jdone = int(hb[hdr + 4]);
        est_out = hb[hdr];
        for (int i = 0; i <= jdone && i <= m; ++i)
            for (int k = 0; k < jdone; ++k) H[size_t(i) * m + k] = hb[size_t(i) * m + k];
        for (int i = 0; i <= jdone; ++i) gv[i] = hb[(m + 1) * m + 2 * m + i];
        return CSDYN_OK;
    };
    int iters = 0, restarts = 0;
    bool conv = beta0 <= tol;
    double est = beta0, beta = beta0;
    while (!conv && iters < maxit) {
        CSD_TRY(Vec<T>::copy(V, r, n, s));
        CSD_TRY(Vec<T>::scale(V, n, 1.0 / beta, s));
        std::fill(gv.begin(), gv.end(), 0.0);
        gv[0] = beta;
        int jdone = 0;
        if (device_steps > 0) {
            bool stop = false;
            CSD_TRY(cycle_dev(std::min(m, maxit - iters), beta, jdone, stop, est));
            iters += jdone;
            if (stop) conv = true;
        } else {
        // With lookahead, step j + 1 is enqueued before the host waits for
        // step j's numbers (unless the convergence rate so far says step j
        // will be the last), so the device does not idle between steps; a
        // step enqueued past convergence is discarded.
        CSD_TRY(launch_step(0));  // step j is always enqueued when the loop reaches j
        double est_prev = est;
        for (int j = 0; j < m && iters < maxit; ++j) {
            const bool more = j + 1 < m && iters + 1 < maxit;
            const double rate = j > 0 && est_prev > 0 ? est / est_prev : 1.0;
            bool ahead = false;
            if (lookahead && more && est * rate > tol) {
                CSD_TRY(launch_step(j + 1));
                ahead = true;
            }
            CSD_HIP(hipEventSynchronize(rb->ev[j % 2]));
            const T *h1 = static_cast<const T *>(rb->buf[j % 2]);
            for (int i = 0; i <= j; ++i)
                H[size_t(i) * m + j] = orth == 0 ? double(h1[i]) : double(h1[i]) + double(h1[kRedStride + i]);
            const double ww = double(h1[kRedStride - 1]);
            const double nn = double(h1[nred * kRedStride - 1]);
            const double hn = std::sqrt(std::max(nn, 0.0));
            H[size_t(j + 1) * m + j] = hn;
            ++iters;
            jdone = j + 1;
            if (!std::isfinite(hn) || !std::isfinite(ww)) { set_error("gmres: non-finite Arnoldi vector"); return CSDYN_EBREAKDOWN; }
            for (int i = 0; i < j; ++i) {
                const double a = H[size_t(i) * m + j], c = H[size_t(i + 1) * m + j];
                H[size_t(i) * m + j] = cs[i] * a + sn[i] * c;
                H[size_t(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
            }
            const double a = H[size_t(j) * m + j], c = H[size_t(j + 1) * m + j];
            const double den = std::hypot(a, c);
            cs[j] = a / den;
            sn[j] = c / den;
            H[size_t(j) * m + j] = den;
            H[size_t(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            est_prev = est;
            est = std::fabs(gv[j + 1]);
            const bool happy = hn <= 1e-14 * std::sqrt(ww);
            if (est <= tol || happy) { conv = true; break; }
            if (!more) break;
            if (!ahead) CSD_TRY(launch_step(j + 1));
        }
        }
        for (int i = jdone - 1; i >= 0; --i) {
            double acc = gv[i];
            for (int k = i + 1; k < jdone; ++k) acc -= H[size_t(i) * m + k] * yv[k];
            yv[i] = acc / H[size_t(i) * m + i];
        }
        if (flexible) {
            CSD_TRY(Vec<T>::lincomb(x, Z, n, jdone, yv.data(), s));
        } else {
            CSD_TRY(Vec<T>::zero(tmp, n, s));
            CSD_TRY(Vec<T>::lincomb(tmp, V, n, jdone, yv.data(), s));
            if (M) CSD_TRY(apply_M(tmp, z));
            else CSD_TRY(Vec<T>::copy(z, tmp, n, s));
            CSD_TRY(Vec<T>::axpby(1.0, z, 1.0, x, n, s));
        }
        CSD_TRY(apply_A(x, tmp));
        CSD_TRY(Vec<T>::copy(r, b, n, s));
        CSD_TRY(Vec<T>::axpby(-1.0, tmp, 1.0, r, n, s));
        CSD_TRY(norm(r, beta, s));
        if (!conv) ++restarts;
    }
    res.iters = iters;
    res.restarts = restarts;
    res.relres_true = beta0 > 0 ? beta / beta0 : 0.0;
    res.relres_est = beta0 > 0 ? est / beta0 : 0.0;
    res.res0 = beta0;
    res.res_true = beta;
    res.bnorm = bnorm;
    res.converged = conv;
    return conv ? CSDYN_OK : CSDYN_ENOTCONV;
}

template struct Gmres<double>;
template struct Gmres<float>;

}  // namespace csd
