// 3x3x3 convolutions on channels-last BF16 tensors with FP32 accumulation on
// the matrix cores, their data and weight gradients, pooling / up-sampling,
// and Adam: the kernels of the learned initial guess.
//
// Tensor layout: [batch][d][h][w][c8] with c8 = round_up(c, 8) and the padded
// channels zero, so every 8-channel group is one 16-byte load.  Weights are
// FP32 [cout][27][cin] (tap t = 9 (dz+1) + 3 (dy+1) + (dx+1)); the kernels use
// packed BF16 copies:
//   wf [round_up(cout,16)][kpad],  k = t*cin8 + c            (forward)
//   wb [round_up(cin,16)][kbpad],  k = t*cout8 + c, W[c][26-t][row]  (data gradient)
// with kpad = round_up(27*cin8, 32) and zeros in every pad position.
//
// Forward and data gradient are one implicit GEMM (M = voxels, N = output
// channels, K = 27 x input channels) on 16x16x32 BF16 MFMA tiles: the data
// gradient is the forward convolution of dY with the flipped, transposed
// weights.  The weight gradient is a GEMM over voxels (M = cout, N = 27 cin,
// K = voxels) with per-split FP32 partials summed in a fixed order.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <type_traits>

#include "common.h"
#include "conv.h"
#include "profile.h"

namespace csd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ inline uint16_t f2bf(float f) {  // round to nearest, ties to even
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float(uint32_t(b) << 16); }

__device__ inline f32x4 mfma(u32x4 a, u32x4 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8, a), __builtin_bit_cast(bf16x8, b), c,
                                                   0, 0, 0);
}

struct Vox {
    int p, d, h, w;
};
__device__ inline Vox decode(int64_t v, const ConvDims &a) {
    Vox o;
    o.w = int(v % a.w);
    int64_t t = v / a.w;
    o.h = int(t % a.h);
    t /= a.h;
    o.d = int(t % a.d);
    o.p = int(t / a.d);
    return o;
}

// --------------------------------------------------------------- forward
// One workgroup: 4 waves x (16 MF voxels) x all 16 NB output channels.  The
// weights of each 32-wide K slab are staged once per workgroup in LDS (double
// buffered) and shared by the four waves; the input fragments come straight
// from the channels-last tensor (16 bytes per lane).
constexpr int kFwSW = 32 + 8;  // LDS row stride of a weight slab (16-bit elements)

template <int NB, int MF>
__global__ __launch_bounds__(256) void k_conv_fwd(ConvDims a, const uint16_t *__restrict__ x,
                                                  const uint16_t *__restrict__ wf, const float *__restrict__ bias,
                                                  const uint16_t *__restrict__ res, const uint16_t *__restrict__ mask,
                                                  int relu, uint16_t *__restrict__ y, float *__restrict__ y32) {
    __shared__ __align__(16) uint16_t sW[2][16 * NB * kFwSW];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int r = lane & 15, g = lane >> 4;
    const int64_t base = (int64_t(blockIdx.x) * 4 + wave) * (16 * MF);
    Vox vx[MF];
    bool ok[MF];
#pragma unroll
    for (int f = 0; f < MF; ++f) {
        const int64_t v = base + f * 16 + r;
        ok[f] = v < a.nvox;
        vx[f] = decode(ok[f] ? v : 0, a);
    }
    f32x4 acc[MF][NB];
#pragma unroll
    for (int f = 0; f < MF; ++f)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) acc[f][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
    // slab loader: 16 NB rows x 32 k = 4 NB 16-byte pieces
    auto stage = [&](int buf, int k0) {
        for (int e = tid; e < 64 * NB; e += 256) {
            const int row = e >> 2, piece = e & 3;
            *reinterpret_cast<u32x4 *>(&sW[buf][row * kFwSW + 8 * piece]) =
                *reinterpret_cast<const u32x4 *>(wf + size_t(row) * a.kpad + k0 + 8 * piece);
        }
    };
    const int nk = a.kpad / 32;
    stage(0, 0);
    __syncthreads();
    for (int kc = 0; kc < nk; ++kc) {
        const int buf = kc & 1;
        if (kc + 1 < nk) stage(buf ^ 1, (kc + 1) * 32);  // next slab, read only after the barrier below
        const int k = kc * 32 + 8 * g;
        const int tap = k / a.ci8, c = k - tap * a.ci8;
        const int dz = tap / 9 - 1, dy = (tap / 3) % 3 - 1, dx = tap % 3 - 1;
        u32x4 af[MF];
#pragma unroll
        for (int f = 0; f < MF; ++f) {
            const int d = vx[f].d + dz, h = vx[f].h + dy, w = vx[f].w + dx;
            const bool in = ok[f] && tap < 27 && d >= 0 && d < a.d && h >= 0 && h < a.h && w >= 0 && w < a.w;
            af[f] = u32x4{0u, 0u, 0u, 0u};
            if (in) {
                const int64_t src = ((int64_t(vx[f].p) * a.d + d) * a.h + h) * a.w + w;
                af[f] = *reinterpret_cast<const u32x4 *>(x + src * a.ci8 + c);
            }
        }
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const u32x4 bf = *reinterpret_cast<const u32x4 *>(&sW[buf][(nb * 16 + r) * kFwSW + 8 * g]);
#pragma unroll
            for (int f = 0; f < MF; ++f) acc[f][nb] = mfma(af[f], bf, acc[f][nb]);
        }
        __syncthreads();  // slab kc consumed by every wave; slab kc+1 complete
    }

#pragma unroll
    for (int f = 0; f < MF; ++f)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int64_t v = base + f * 16 + 4 * g + i;
            if (v >= a.nvox) continue;
#pragma unroll
            for (int nb = 0; nb < NB; ++nb) {
                const int co = nb * 16 + r;
                float val = 0.f;
                if (co < a.co) {
                    val = acc[f][nb][i];
                    if (bias) val += bias[co];
                    if (res) val += bf2f(res[v * a.co8 + co]);
                    if (relu) val = fmaxf(val, 0.f);
                    if (mask && !(bf2f(mask[v * a.co8 + co]) > 0.f)) val = 0.f;
                }
                if (y && co < a.co8) y[v * a.co8 + co] = f2bf(val);
                if (y32 && co < a.co) y32[v * a.co + co] = val;
            }
        }
}

// -------------------------------------------------------- weight gradient
// dW[co][k] = sum_v dY[v][co] X[v + off(t(k))][c(k)]: a GEMM over voxels.  One
// workgroup owns all output-channel rows x 64 consecutive K columns and sums a
// strided set of 64-voxel chunks.  Each chunk is staged through LDS transposed
// ([row][voxel], voxels contiguous), so every MFMA operand is one 16-byte LDS
// read; wave w takes column fragment w and all row fragments.
constexpr int kBwVC = 64;          // voxels per chunk
constexpr int kBwSA = kBwVC + 8;   // LDS row stride in 16-bit elements (spreads banks)

template <int NRF>
__global__ __launch_bounds__(256) void k_conv_bwdw(ConvDims a, const uint16_t *__restrict__ x,
                                                   const uint16_t *__restrict__ dy, int kcols, int nsplit,
                                                   float *__restrict__ partial) {
    constexpr int COPAD = 16 * NRF;
    __shared__ __align__(16) uint16_t sA[COPAD * kBwSA];  // dY^T  [co][v]
    __shared__ __align__(16) uint16_t sB[64 * kBwSA];     // X_k^T [col][v]
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, r = lane & 15, g = lane >> 4;
    const int colbase = blockIdx.x * 64;
    // rows beyond the tensor's channels stay zero
    for (int e = tid; e < (COPAD - a.co8) * kBwSA; e += 256) sA[a.co8 * kBwSA + e] = 0;
    f32x4 acc[NRF];
    for (int f = 0; f < NRF; ++f) acc[f] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int cgA = a.co8 / 8;  // 8-channel groups of dY
    const int64_t nchunks = (a.nvox + kBwVC - 1) / kBwVC;
    for (int64_t chunk = blockIdx.z; chunk < nchunks; chunk += nsplit) {
        const int64_t v0 = chunk * kBwVC;
        for (int e = tid; e < kBwVC * cgA; e += 256) {
            const int vv = e / cgA, cg = e - vv * cgA;
            const int64_t v = v0 + vv;
            u32x4 q = u32x4{0u, 0u, 0u, 0u};
            if (v < a.nvox) q = *reinterpret_cast<const u32x4 *>(dy + v * a.co8 + cg * 8);
            for (int h = 0; h < 4; ++h) {
                sA[(cg * 8 + 2 * h) * kBwSA + vv] = uint16_t(q[h] & 0xFFFFu);
                sA[(cg * 8 + 2 * h + 1) * kBwSA + vv] = uint16_t(q[h] >> 16);
            }
        }
        for (int e = tid; e < kBwVC * 8; e += 256) {
            const int vv = e >> 3, cg = e & 7;
            const int col0 = colbase + cg * 8;
            const int tap = col0 / a.ci8, c = col0 - tap * a.ci8;
            const int64_t v = v0 + vv;
            u32x4 q = u32x4{0u, 0u, 0u, 0u};
            if (v < a.nvox && tap < 27) {
                const Vox o = decode(v, a);
                const int d = o.d + tap / 9 - 1, hh = o.h + (tap / 3) % 3 - 1, w = o.w + tap % 3 - 1;
                if (d >= 0 && d < a.d && hh >= 0 && hh < a.h && w >= 0 && w < a.w)
                    q = *reinterpret_cast<const u32x4 *>(
                        x + (((int64_t(o.p) * a.d + d) * a.h + hh) * a.w + w) * a.ci8 + c);
            }
            for (int h = 0; h < 4; ++h) {
                sB[(cg * 8 + 2 * h) * kBwSA + vv] = uint16_t(q[h] & 0xFFFFu);
                sB[(cg * 8 + 2 * h + 1) * kBwSA + vv] = uint16_t(q[h] >> 16);
            }
        }
        __syncthreads();
        for (int ks = 0; ks < kBwVC / 32; ++ks) {
            const int vo = ks * 32 + 8 * g;
            const u32x4 B = *reinterpret_cast<const u32x4 *>(&sB[(wave * 16 + r) * kBwSA + vo]);
            for (int f = 0; f < NRF; ++f) {
                const u32x4 A = *reinterpret_cast<const u32x4 *>(&sA[(f * 16 + r) * kBwSA + vo]);
                acc[f] = mfma(A, B, acc[f]);
            }
        }
        __syncthreads();
    }
    float *out = partial + size_t(blockIdx.z) * COPAD * kcols;
    for (int f = 0; f < NRF; ++f)
        for (int i = 0; i < 4; ++i)
            out[size_t(f * 16 + 4 * g + i) * kcols + colbase + wave * 16 + r] = acc[f][i];
}

// dW[co][t][c] = sum over splits, in split order.
__global__ void k_bwdw_reduce(ConvDims a, const float *__restrict__ partial, int kcols, int copad, int nsplit,
                              float *__restrict__ dw) {
    const int64_t n = int64_t(a.co) * 27 * a.ci;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int c = int(e % a.ci), t = int((e / a.ci) % 27), co = int(e / (27 * int64_t(a.ci)));
    const size_t off = size_t(co) * kcols + size_t(t) * a.ci8 + c;
    float s = 0.f;
    for (int z = 0; z < nsplit; ++z) s += partial[size_t(z) * copad * kcols + off];
    dw[e] = s;
}

// Bias gradient: block partial sums over voxel ranges, then a fixed-order sum.
constexpr int kColsumBlocks = 512;
__global__ __launch_bounds__(256) void k_colsum(int64_t nvox, int c8, const uint16_t *__restrict__ t,
                                                float *__restrict__ partial) {
    __shared__ float red[256];
    const int nsub = 256 / c8;
    const int c = threadIdx.x % c8, sub = threadIdx.x / c8;
    const int64_t per = (nvox + gridDim.x - 1) / gridDim.x;
    const int64_t v0 = int64_t(blockIdx.x) * per, v1 = std::min<int64_t>(nvox, v0 + per);
    float s = 0.f;
    if (sub < nsub)
        for (int64_t v = v0 + sub; v < v1; v += nsub) s += bf2f(t[v * c8 + c]);
    red[threadIdx.x] = s;
    __syncthreads();
    if (threadIdx.x < c8) {
        float tot = 0.f;
        for (int q = 0; q < nsub; ++q) tot += red[q * c8 + threadIdx.x];
        partial[size_t(blockIdx.x) * c8 + threadIdx.x] = tot;
    }
}
__global__ void k_colsum_final(int nblk, int c8, int c, const float *__restrict__ partial, float *__restrict__ out) {
    const int j = threadIdx.x;
    if (j >= c) return;
    float s = 0.f;
    for (int b = 0; b < nblk; ++b) s += partial[size_t(b) * c8 + j];
    out[j] = s;
}

// ------------------------------------------------------------ weight packing
__global__ void k_pack(ConvDims a, const float *__restrict__ w, uint16_t *__restrict__ wf, int copad,
                       uint16_t *__restrict__ wb, int cipad, int kbpad) {
    const int64_t nf = int64_t(copad) * a.kpad, nb = int64_t(cipad) * kbpad;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (wf && e < nf) {
        const int row = int(e / a.kpad), k = int(e % a.kpad);
        const int t = k / a.ci8, c = k % a.ci8;
        wf[e] = (row < a.co && t < 27 && c < a.ci) ? f2bf(w[(size_t(row) * 27 + t) * a.ci + c]) : uint16_t(0);
    }
    if (wb && e < nb) {
        const int row = int(e / kbpad), k = int(e % kbpad);
        const int t = k / a.co8, c = k % a.co8;  // c: forward output channel
        wb[e] = (row < a.ci && t < 27 && c < a.co) ? f2bf(w[(size_t(c) * 27 + (26 - t)) * a.ci + row]) : uint16_t(0);
    }
}

// ---------------------------------------------------- pooling / up-sampling
// dst (coarse) = scale * mean of the 8 children of src (fine) [+ add] [masked]
__global__ void k_pool(int nb, int d, int h, int w, int c8, const uint16_t *__restrict__ src, float scale,
                       const uint16_t *__restrict__ add, const uint16_t *__restrict__ mask,
                       uint16_t *__restrict__ dst) {
    const int64_t n = int64_t(nb) * d * h * w * c8;
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int c = int(e % c8);
    int64_t v = e / c8;
    const int i = int(v % w); v /= w;
    const int j = int(v % h); v /= h;
    const int k = int(v % d);
    const int64_t p = v / d;
    float s = 0.f;
    for (int dz = 0; dz < 2; ++dz)
        for (int dy = 0; dy < 2; ++dy)
            for (int dx = 0; dx < 2; ++dx)
                s += bf2f(src[((((p * 2 * d) + 2 * k + dz) * 2 * h + 2 * j + dy) * 2 * w + 2 * i + dx) * c8 + c]);
    float val = scale * (s * 0.125f);
    if (add) val += bf2f(add[e]);
    if (mask && !(bf2f(mask[e]) > 0.f)) val = 0.f;
    dst[e] = f2bf(val);
}

// dst (fine) = scale * parent of src (coarse) [+ add] [masked]
__global__ void k_up(int nb, int d, int h, int w, int c8, const uint16_t *__restrict__ src, float scale,
                     const uint16_t *__restrict__ add, const uint16_t *__restrict__ mask,
                     uint16_t *__restrict__ dst) {
    const int64_t n = int64_t(nb) * d * h * w * c8;  // fine sizes
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const int c = int(e % c8);
    int64_t v = e / c8;
    const int i = int(v % w); v /= w;
    const int j = int(v % h); v /= h;
    const int k = int(v % d);
    const int64_t p = v / d;
    float val = scale * bf2f(src[(((p * (d / 2) + k / 2) * (h / 2) + j / 2) * (w / 2) + i / 2) * c8 + c]);
    if (add) val += bf2f(add[e]);
    if (mask && !(bf2f(mask[e]) > 0.f)) val = 0.f;
    dst[e] = f2bf(val);
}

// ------------------------------------------------------------------- Adam
__global__ void k_adam(float *__restrict__ p, const float *__restrict__ gr, float *__restrict__ m,
                       float *__restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float c1, float c2) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= n) return;
    const float g = gr[e];
    const float mm = b1 * m[e] + (1.f - b1) * g;
    const float vv = b2 * v[e] + (1.f - b2) * g * g;
    m[e] = mm;
    v[e] = vv;
    p[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// --------------------------------------------------------------- launchers
static inline int rup(int x, int m) { return (x + m - 1) / m * m; }

int32_t conv_dims(const csdyn_conv_shape *s, ConvDims &a) {
    if (!s) { set_error("conv: null shape"); return CSDYN_EINVAL; }
    if (s->batch < 1 || s->d < 1 || s->h < 1 || s->w < 1 || s->cin < 1 || s->cout < 1 || s->cin > 1024 ||
        s->cout > 128) {
        set_error("conv: bad shape (batch %d, %dx%dx%d, cin %d, cout %d; cout <= 128, cin <= 1024)", s->batch, s->d,
                  s->h, s->w, s->cin, s->cout);
        return CSDYN_EINVAL;
    }
    a.nb = s->batch; a.d = s->d; a.h = s->h; a.w = s->w;
    a.ci = s->cin; a.co = s->cout;
    a.ci8 = rup(a.ci, 8); a.co8 = rup(a.co, 8);
    a.kpad = rup(27 * a.ci8, 32);
    a.nvox = int64_t(a.nb) * a.d * a.h * a.w;
    return CSDYN_OK;
}

// the data-gradient convolution: input channels cout, output channels cin
static ConvDims transposed(const ConvDims &a) {
    ConvDims b = a;
    b.ci = a.co; b.co = a.ci; b.ci8 = a.co8; b.co8 = a.ci8;
    b.kpad = rup(27 * b.ci8, 32);
    return b;
}

int32_t conv_fwd_launch(const ConvDims &a, const uint16_t *x, const uint16_t *wf, const float *bias,
                        const uint16_t *res, const uint16_t *mask, int relu, uint16_t *y, float *y32, hipStream_t s,
                        const char *name) {
    const int nbk = rup(a.co, 16) / 16;
    ProfScope ps(name, a.nvox, double(a.nvox) * 2.0 * (a.ci + a.co), s, 2.0 * a.nvox * a.co * 27.0 * a.ci);
    // four row fragments per wave (256 voxels per workgroup), two for the widest outputs
    auto go = [&](auto nb_c, auto mf_c) {
        constexpr int NB = decltype(nb_c)::value, MF = decltype(mf_c)::value;
        const dim3 grid(unsigned((a.nvox + 64 * MF - 1) / (64 * MF)));
        hipLaunchKernelGGL((k_conv_fwd<NB, MF>), grid, dim3(256), 0, s, a, x, wf, bias, res, mask, relu, y, y32);
    };
    using std::integral_constant;
#define CONV_CASE(NB, MF)                                             \
    case NB:                                                          \
        go(integral_constant<int, NB>(), integral_constant<int, MF>()); \
        break;
    switch (nbk) {
        CONV_CASE(1, 4) CONV_CASE(2, 4) CONV_CASE(3, 4) CONV_CASE(4, 4) CONV_CASE(5, 2) CONV_CASE(6, 2)
        CONV_CASE(7, 2) CONV_CASE(8, 2)
        default: set_error("conv: cout %d unsupported", a.co); return CSDYN_EINVAL;
    }
#undef CONV_CASE
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

int32_t conv_bwd_data_launch(const ConvDims &a, const uint16_t *dy, const uint16_t *wb, const uint16_t *mask,
                             uint16_t *dx, hipStream_t s) {
    const ConvDims b = transposed(a);
    if (b.co > 128) { set_error("conv bwd_data: cin %d > 128 unsupported", a.ci); return CSDYN_EINVAL; }
    return conv_fwd_launch(b, dy, wb, nullptr, nullptr, mask, 0, dx, nullptr, s, "conv_bwd_data");
}

struct BwdwPlan {
    int nrf, copad, colblocks, kcols, nsplit;
    size_t partial_bytes, colsum_bytes;
};
static BwdwPlan bwdw_plan(const ConvDims &a) {
    BwdwPlan p;
    p.copad = rup(a.co8, 16);
    p.nrf = p.copad / 16;
    p.kcols = rup(27 * a.ci8, 64);
    p.colblocks = p.kcols / 64;
    const int64_t nchunks = (a.nvox + kBwVC - 1) / kBwVC;
    int64_t ns = std::max<int64_t>(1, 2048 / p.colblocks);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, nchunks / 4));
    const size_t per = size_t(p.copad) * p.kcols * sizeof(float);
    ns = std::min<int64_t>(ns, std::max<int64_t>(1, int64_t((size_t(256) << 20) / per)));
    p.nsplit = int(ns);
    p.partial_bytes = per * size_t(p.nsplit);
    p.colsum_bytes = size_t(kColsumBlocks) * a.co8 * sizeof(float);
    return p;
}

size_t conv_bwd_weight_ws(const ConvDims &a) {
    const BwdwPlan p = bwdw_plan(a);
    Carver c(nullptr);
    c.take<float>(p.partial_bytes / sizeof(float));
    c.take<float>(p.colsum_bytes / sizeof(float));
    return c.off + 256;
}

int32_t conv_bwd_weight_launch(const ConvDims &a, const uint16_t *x, const uint16_t *dy, float *dw, float *db,
                               void *ws, size_t ws_bytes, hipStream_t s) {
    const BwdwPlan p = bwdw_plan(a);
    if (ws_bytes < conv_bwd_weight_ws(a)) { set_error("conv bwd_weight: workspace too small"); return CSDYN_ENOMEM; }
    Carver c(ws);
    float *partial = c.take<float>(p.partial_bytes / sizeof(float));
    float *colsum = c.take<float>(p.colsum_bytes / sizeof(float));
    {
        ProfScope ps("conv_bwd_weight", a.nvox, double(a.nvox) * 2.0 * (a.ci8 + a.co8), s,
                     2.0 * a.nvox * a.co * 27.0 * a.ci);
        const dim3 grid(p.colblocks, 1, p.nsplit);
#define BWDW_CASE(NRF)                                                                                 \
    case NRF:                                                                                          \
        hipLaunchKernelGGL(k_conv_bwdw<NRF>, grid, dim3(256), 0, s, a, x, dy, p.kcols, p.nsplit, partial); \
        break;
        switch (p.nrf) {
            BWDW_CASE(1) BWDW_CASE(2) BWDW_CASE(3) BWDW_CASE(4) BWDW_CASE(5) BWDW_CASE(6) BWDW_CASE(7) BWDW_CASE(8)
            default: set_error("conv bwd_weight: cout %d unsupported", a.co); return CSDYN_EINVAL;
        }
#undef BWDW_CASE
        CSD_HIP(hipGetLastError());
        const int64_t n = int64_t(a.co) * 27 * a.ci;
        hipLaunchKernelGGL(k_bwdw_reduce, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a, partial, p.kcols,
                           p.copad, p.nsplit, dw);
        CSD_HIP(hipGetLastError());
    }
    if (db) {
        hipLaunchKernelGGL(k_colsum, dim3(kColsumBlocks), dim3(256), 0, s, a.nvox, a.co8, dy, colsum);
        hipLaunchKernelGGL(k_colsum_final, dim3(1), dim3(128), 0, s, kColsumBlocks, a.co8, a.co, colsum, db);
        CSD_HIP(hipGetLastError());
    }
    return CSDYN_OK;
}

void conv_packed_sizes(const ConvDims &a, int64_t &wf_elems, int64_t &wb_elems) {
    const ConvDims b = transposed(a);
    wf_elems = int64_t(rup(a.co, 16)) * a.kpad;
    wb_elems = int64_t(rup(a.ci, 16)) * b.kpad;
}

int32_t conv_pack_launch(const ConvDims &a, const float *w, uint16_t *wf, uint16_t *wb, hipStream_t s) {
    const ConvDims b = transposed(a);
    int64_t nf, nbk;
    conv_packed_sizes(a, nf, nbk);
    const int64_t n = std::max(nf, nbk);
    hipLaunchKernelGGL(k_pack, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, a, w, wf, rup(a.co, 16), wb,
                       rup(a.ci, 16), b.kpad);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

int32_t pool_launch(int nb, int d, int h, int w, int c8, const uint16_t *src, float scale, const uint16_t *add,
                    const uint16_t *mask, uint16_t *dst, hipStream_t s) {
    const int64_t n = int64_t(nb) * d * h * w * c8;
    ProfScope ps("pool", n, double(n) * 2.0 * (8 + 1 + (add ? 1 : 0) + (mask ? 1 : 0)), s);
    hipLaunchKernelGGL(k_pool, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, nb, d, h, w, c8, src, scale, add,
                       mask, dst);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

int32_t up_launch(int nb, int d, int h, int w, int c8, const uint16_t *src, float scale, const uint16_t *add,
                  const uint16_t *mask, uint16_t *dst, hipStream_t s) {
    const int64_t n = int64_t(nb) * d * h * w * c8;
    ProfScope ps("up", n, double(n) * 2.0 * (1.125 + (add ? 1 : 0) + (mask ? 1 : 0)), s);
    hipLaunchKernelGGL(k_up, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, nb, d, h, w, c8, src, scale, add,
                       mask, dst);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

int32_t adam_launch(float *p, const float *g, float *m, float *v, int64_t n, int32_t step, float lr, float b1,
                    float b2, float eps, hipStream_t s) {
    const float c1 = float(1.0 - std::pow(double(b1), step)), c2 = float(1.0 - std::pow(double(b2), step));
    hipLaunchKernelGGL(k_adam, dim3(unsigned((n + 255) / 256)), dim3(256), 0, s, p, g, m, v, n, lr, b1, b2, eps, c1,
                       c2);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

}  // namespace csd

using namespace csd;

extern "C" int32_t csdyn_conv3d_sizes(const csdyn_conv_shape *s, int64_t *wf_elems, int64_t *wb_elems,
                                      size_t *bwd_weight_ws_bytes) {
    clear_error();
    ConvDims a;
    CSD_TRY(conv_dims(s, a));
    int64_t nf, nb;
    conv_packed_sizes(a, nf, nb);
    if (wf_elems) *wf_elems = nf;
    if (wb_elems) *wb_elems = nb;
    if (bwd_weight_ws_bytes) *bwd_weight_ws_bytes = conv_bwd_weight_ws(a);
    return CSDYN_OK;
}

extern "C" int32_t csdyn_conv3d_pack(const csdyn_conv_shape *s, const float *w, uint16_t *wf, uint16_t *wb,
                                     void *stream) {
    clear_error();
    ConvDims a;
    CSD_TRY(conv_dims(s, a));
    if (!w || (!wf && !wb)) { set_error("csdyn_conv3d_pack: null pointer"); return CSDYN_EINVAL; }
    return conv_pack_launch(a, w, wf, wb, (hipStream_t)stream);
}

extern "C" int32_t csdyn_conv3d_fwd(const csdyn_conv_shape *s, const uint16_t *x, const uint16_t *wf,
                                    const float *bias, const uint16_t *residual, int32_t relu, uint16_t *y,
                                    float *y32, void *stream) {
    clear_error();
    ConvDims a;
    CSD_TRY(conv_dims(s, a));
    if (!x || !wf || (!y && !y32)) { set_error("csdyn_conv3d_fwd: null pointer"); return CSDYN_EINVAL; }
    return conv_fwd_launch(a, x, wf, bias, residual, nullptr, relu ? 1 : 0, y, y32, (hipStream_t)stream,
                           "conv_fwd");
}

extern "C" int32_t csdyn_conv3d_bwd_data(const csdyn_conv_shape *s, const uint16_t *dy, const uint16_t *wb,
                                         const uint16_t *mask, uint16_t *dx, void *stream) {
    clear_error();
    ConvDims a;
    CSD_TRY(conv_dims(s, a));
    if (!dy || !wb || !dx) { set_error("csdyn_conv3d_bwd_data: null pointer"); return CSDYN_EINVAL; }
    return conv_bwd_data_launch(a, dy, wb, mask, dx, (hipStream_t)stream);
}

extern "C" int32_t csdyn_conv3d_bwd_weight(const csdyn_conv_shape *s, const uint16_t *x, const uint16_t *dy,
                                           float *dw, float *db, void *ws, size_t ws_bytes, void *stream) {
    clear_error();
    ConvDims a;
    CSD_TRY(conv_dims(s, a));
    if (!x || !dy || !dw || !ws) { set_error("csdyn_conv3d_bwd_weight: null pointer"); return CSDYN_EINVAL; }
    return conv_bwd_weight_launch(a, x, dy, dw, db, ws, ws_bytes, (hipStream_t)stream);
}

extern "C" int32_t csdyn_adam_step(float *param, const float *grad, float *m, float *v, int64_t n, int32_t step,
                                   float lr, float beta1, float beta2, float eps, void *stream) {
    clear_error();
    if (!param || !grad || !m || !v || n < 0 || step < 1) {
        set_error("csdyn_adam_step: bad argument");
        return CSDYN_EINVAL;
    }
    if (n == 0) return CSDYN_OK;
    return adam_launch(param, grad, m, v, n, step, lr, beta1, beta2, eps, (hipStream_t)stream);
}
