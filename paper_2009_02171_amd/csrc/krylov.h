// Restarted GMRES / FGMRES engine (Sec. 3.3) on device vectors, with the
// operator and preconditioner passed as callbacks.  Used by csdyn_gmres_solve
// (FP64) and by the coarse solve inside the two-level preconditioner.
#pragma once

#include <functional>
#include <vector>

#include "common.h"

namespace csd {

constexpr int kRedStride = 33;  // 32 dot products + 1 self product per block
constexpr int kMaxBlocks = 1024;  // blocks of the reduction kernels
// Entries of a reduction partial buffer: partial[q * kMaxBlocks + block],
// q < kRedStride, whatever the vector length.
constexpr size_t kPartialElems = size_t(kMaxBlocks) * kRedStride;
constexpr int kMaxRestart = 64;

template <class T>
using DevFn = std::function<int32_t(const T *in, T *out, hipStream_t s)>;

// Vector kernels (deterministic: fixed block decomposition, fixed reduction order).
template <class T>
struct Vec {
    static int nblocks(int64_t n);
    // out[q] = V_q . w (q < cnt), out[32] = w . w; partial has nblocks*kRedStride entries
    static int32_t mdot(const T *V, int64_t n, int cnt, const T *w, T *partial, T *out, hipStream_t s);
    // w -= sum_q h[q] V_q (h on device), then out[32] = w . w
    static int32_t mupdate(T *w, const T *V, int64_t n, int cnt, const T *h, T *partial, T *out, hipStream_t s);
    // the update pass alone: partial[32][block] = each block's part of ||w||^2, left for the caller to sum
    static int32_t mupdate_blocks(T *w, const T *V, int64_t n, int cnt, const T *h, T *partial, hipStream_t s);
    // w -= sum_q h[q] V_q; out[q] = V_q . w_new (q < cnt), out[32] = ||w_new||^2
    static int32_t mupdate_dot(T *w, const T *V, int64_t n, int cnt, const T *h, T *partial, T *out, hipStream_t s);
    static int32_t scale(T *w, int64_t n, double a, hipStream_t s);
    // y = a*x + b*y
    static int32_t axpby(double a, const T *x, double b, T *y, int64_t n, hipStream_t s);
    // x += sum_q c[q] Z_q
    static int32_t lincomb(T *x, const T *Z, int64_t n, int cnt, const double *c, hipStream_t s);
    static int32_t copy(T *dst, const T *src, int64_t n, hipStream_t s);
    static int32_t zero(T *x, int64_t n, hipStream_t s);
    // out[0] = sum vol * x_P, out[1] = sum vol  (4-component layout, P = component 3)
    static int32_t pmoments(const T *x, const double *vol, int64_t ncell, T *partial, T *out, hipStream_t s);
    static int32_t padd(T *x, int64_t ncell, double c, hipStream_t s);
    // the pressure components shifted by -mom[0] / mom[1], the moments pmoments left on the device
    static int32_t padd_mean(T *x, int64_t ncell, const T *mom, hipStream_t s);
};

int32_t convert_d2f(const double *x, float *y, int64_t n, hipStream_t s);
int32_t convert_f2d(const float *x, double *y, int64_t n, hipStream_t s);

struct GmresResult {
    int iters = 0, restarts = 0;
    double relres_true = 0, relres_est = 0;
    double res0 = 0, res_true = 0, bnorm = 0;
    bool converged = false;
};

template <class T>
struct Gmres {
    int64_t n = 0;
    int m = 30;
    bool flexible = false;
    int orth = 0;  // 0: classical Gram-Schmidt, 1: with one re-orthogonalisation pass
    // Enqueue Arnoldi step j + 1 before reading back step j (for solves whose
    // steps are short device work; a step enqueued past convergence is wasted)
    bool lookahead = false;
    // Phase (profile.h) under which the preconditioner's time is recorded when
    // the solve is timed; -1: the preconditioner records its own phases.
    int m_phase = -1;
    // device_steps = k > 0: the Hessenberg column, Givens rotation and residual
    // estimate of each Arnoldi step are formed on the device, and the host
    // reads the convergence state once per group of k steps, with the next
    // group already enqueued (steps enqueued past convergence are discarded).
    // 0: the host forms them from each step's read-back.
    int device_steps = 0;
    T *V = nullptr, *Z = nullptr, *z = nullptr, *r = nullptr, *tmp = nullptr, *partial = nullptr, *red = nullptr;
    double *gs = nullptr;  // device rotation state (device_steps > 0), gs_elems(m) entries
    // H [(m + 1) x m] (rotated, upper triangular), cs [m], sn [m], g [m + 1],
    // then the header: estimate, stopped, converged, breakdown, steps done.
    static constexpr int gs_elems(int m) { return (m + 1) * m + 3 * m + 1 + 8; }

    static size_t bytes(int64_t n, int m, bool flexible);
    void carve(Carver &c, int64_t n_, int m_, bool flexible_);
    // Solve A x = b to max(atol, rtol * ref) with right preconditioning, ref =
    // ||b - A x0|| (or ||b|| when rhs_relative).
    int32_t solve(const DevFn<T> &A, const DevFn<T> *M, const T *b, T *x, int maxit, double rtol, double atol,
                  hipStream_t s, GmresResult &res, bool rhs_relative = false);
    int32_t norm(const T *v, double &out, hipStream_t s);

   private:
    int32_t fetch(int cnt, std::vector<T> &out, hipStream_t s);
};

}  // namespace csd
