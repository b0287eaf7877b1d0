// Device code of the Krylov vector reductions (Sec. 3.3), shared by the
// GMRES kernels (krylov.hip) and the persistent batched Arnoldi step
// (batched.hip): block-partial multi-dot and multi-update over the basis and
// the fixed-order reduction of the partials.
#pragma once

#include "krylov.h"

namespace csd {

constexpr int kBlk = 256;

template <class T>
__device__ __forceinline__ T wave_sum(T v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    return v;
}

template <class T>
int Vec<T>::nblocks(int64_t n) {
    int64_t b = (n + int64_t(kBlk) * 4 - 1) / (int64_t(kBlk) * 4);
    return int(std::max<int64_t>(1, std::min<int64_t>(kMaxBlocks, b)));
}

// Block sums of the kRedStride accumulators (wavefront shuffles, then the
// waves in order), written to partial[q][block] (q-major).
template <class T>
__device__ __forceinline__ void block_store(T (&acc)[kRedStride], int cnt_total, T *partial, int b) {
    __shared__ T sm[kBlk / 64][kRedStride];
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
#pragma unroll
    for (int q = 0; q < kRedStride; ++q) {
        if (q < cnt_total || q == kRedStride - 1) {
            const T v = wave_sum(acc[q]);
            if (lane == 0) sm[wv][q] = v;
        }
    }
    __syncthreads();
    if (threadIdx.x < kRedStride) {
        T s = 0;
        for (int w = 0; w < kBlk / 64; ++w) s += sm[w][threadIdx.x];
        partial[size_t(threadIdx.x) * kMaxBlocks + b] = s;
    }
}

// 16-byte vectors of T: the orthogonalisation kernels stream the basis with
// one 16-byte load per vector and element pair (FP64) or quad (FP32); every
// vector length is a multiple of 24, so the width always divides it.
template <class T>
struct Vec16;
template <>
struct Vec16<double> {
    using type = double2;
    static constexpr int W = 2;
    __device__ static double get(const double2 &v, int e) { return e == 0 ? v.x : v.y; }
    __device__ static void set(double2 &v, int e, double a) { (e == 0 ? v.x : v.y) = a; }
};
template <>
struct Vec16<float> {
    using type = float4;
    static constexpr int W = 4;
    __device__ static float get(const float4 &v, int e) { return e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w; }
    __device__ static void set(float4 &v, int e, float a) { (e == 0 ? v.x : e == 1 ? v.y : e == 2 ? v.z : v.w) = a; }
};

// Block b of nb (kBlk threads) of the multi-dot: partial[q][b] = its part of
// V_q . w (q < cnt) and of w . w (q = 32).
template <class T>
__device__ __forceinline__ void mdot_block(const T *__restrict__ V, int64_t n, int cnt, const T *__restrict__ w,
                                           T *__restrict__ partial, int b, int nb) {
    using VT = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    T acc[kRedStride];
#pragma unroll
    for (int q = 0; q < kRedStride; ++q) acc[q] = 0;
    const int64_t nv = n / W, stride = int64_t(nb) * kBlk;
    const VT *Vv = reinterpret_cast<const VT *>(V);
    const VT *wv4 = reinterpret_cast<const VT *>(w);
    for (int64_t i = int64_t(b) * kBlk + threadIdx.x; i < nv; i += stride) {
        const VT wv = wv4[i];
#pragma unroll
        for (int q = 0; q < kRedStride - 1; ++q)
            if (q < cnt) {
                const VT v = Vv[int64_t(q) * nv + i];
#pragma unroll
                for (int e = 0; e < W; ++e) acc[q] += Vec16<T>::get(v, e) * Vec16<T>::get(wv, e);
            }
#pragma unroll
        for (int e = 0; e < W; ++e) acc[kRedStride - 1] += Vec16<T>::get(wv, e) * Vec16<T>::get(wv, e);
    }
    block_store(acc, cnt, partial, b);
}

// Block b of nb of the multi-update w -= sum_q h[q] V_q, partial[32][b] = its
// part of ||w||^2.
template <class T>
__device__ __forceinline__ void mupdate_block(T *__restrict__ w, const T *__restrict__ V, int64_t n, int cnt,
                                              const T *__restrict__ h, T *__restrict__ partial, int b, int nb) {
    using VT = typename Vec16<T>::type;
    constexpr int W = Vec16<T>::W;
    T hq[kRedStride - 1];
#pragma unroll
    for (int q = 0; q < kRedStride - 1; ++q) hq[q] = q < cnt ? h[q] : T(0);
    T acc[kRedStride];
#pragma unroll
    for (int q = 0; q < kRedStride; ++q) acc[q] = 0;
    const int64_t nv = n / W, stride = int64_t(nb) * kBlk;
    const VT *Vv = reinterpret_cast<const VT *>(V);
    VT *wv4 = reinterpret_cast<VT *>(w);
    for (int64_t i = int64_t(b) * kBlk + threadIdx.x; i < nv; i += stride) {
        VT wv = wv4[i];
#pragma unroll
        for (int q = 0; q < kRedStride - 1; ++q)
            if (q < cnt) {
                const VT v = Vv[int64_t(q) * nv + i];
#pragma unroll
                for (int e = 0; e < W; ++e) Vec16<T>::set(wv, e, Vec16<T>::get(wv, e) - hq[q] * Vec16<T>::get(v, e));
            }
        wv4[i] = wv;
#pragma unroll
        for (int e = 0; e < W; ++e) acc[kRedStride - 1] += Vec16<T>::get(wv, e) * Vec16<T>::get(wv, e);
    }
    block_store(acc, 0, partial, b);
}

// out[q] = sum over blocks b < nb of partial[q][b] for q < cnt and q = 32, in a
// fixed order (one thread per block index, then the block reduction).
// With NT < 1024 threads each wavefront takes the 64-block groups of
// 1024 / NT wavefronts in turn, so the sums are the same, in the same order, as
// with 1024 threads.
template <class T, int NT>
__device__ __forceinline__ void reduce_block(const T *__restrict__ partial, int nb, int cnt, T *__restrict__ out) {
    static_assert(NT % 64 == 0 && 1024 % NT == 0, "workgroup of 64..1024 threads");
    __shared__ T sm[1024 / 64][kRedStride];
    const int lane = threadIdx.x % 64, wv = threadIdx.x / 64;
    for (int vw = wv; vw < 1024 / 64; vw += NT / 64) {
        const int t = vw * 64 + lane;
        T acc[kRedStride];
#pragma unroll
        for (int q = 0; q < kRedStride; ++q) {
            acc[q] = 0;
            if ((q < cnt || q == kRedStride - 1) && t < nb) acc[q] = partial[size_t(q) * kMaxBlocks + t];
        }
#pragma unroll
        for (int q = 0; q < kRedStride; ++q) {
            if (q < cnt || q == kRedStride - 1) {
                const T v = wave_sum(acc[q]);
                if (lane == 0) sm[vw][q] = v;
            }
        }
    }
    __syncthreads();
    if (threadIdx.x < kRedStride && (int(threadIdx.x) < cnt || threadIdx.x == kRedStride - 1)) {
        T s = 0;
        for (int w = 0; w < 1024 / 64; ++w) s += sm[w][threadIdx.x];
        out[threadIdx.x] = s;
    }
}

}  // namespace csd
