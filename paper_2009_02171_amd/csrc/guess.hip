// Initial guesses for the solves of a time march (the paper starts each solve
// from the previous step's solution, Sec. 3.3) and the right-hand side of the
// march that trains and evaluates the learned guess.
//
// csdyn_guess: x_e = 2 x1 - x2 (linear extrapolation); with the network,
// x_n = x_e + sd * net(x1, x2) and d = x_n - x_e.  Residuals come from two
// operator applies by linearity, r_e = b - A x_e and r_n = r_e - A d:
//   mode 1 keeps x_n when ||r_n|| < ||r_e||, else x_e;
//   mode 2 returns x_e + alpha d with alpha = <r_e, A d> / <A d, A d>, the
//          step along the network's correction that minimises the residual
//          (never larger than ||r_e||).
#include <cmath>

#include "krylov.h"
#include "profile.h"

namespace csd {
namespace {

__global__ void k_extrapolate(const double *__restrict__ x1, const double *__restrict__ x2, double *__restrict__ out,
                              int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) out[i] = 2.0 * x1[i] - x2[i];
}

// b = (v + dt f, 0): the vector part of the state plus the forcing, zero scalar part
__global__ void k_march_rhs(const double *__restrict__ v, const double *__restrict__ f, double dt,
                            double *__restrict__ b, int64_t ncell) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; e < 4 * ncell; e += stride)
        b[e] = (e & 3) == 3 ? 0.0 : v[e] + dt * f[e];
}

dim3 grid_of(int64_t n) { return dim3(unsigned(n > 0 ? (n + 255) / 256 < 8192 ? (n + 255) / 256 : 8192 : 1)); }

struct GuessLayout {
    double *bp, *xe, *d, *ad_re, *partial, *red;  // ad_re: [2][n], A d then r_e
};

void guess_layout(Carver &c, int64_t n, GuessLayout &L) {
    L.bp = c.take<double>(n);
    L.xe = c.take<double>(n);
    L.d = c.take<double>(n);
    L.ad_re = c.take<double>(2 * n);
    L.partial = c.take<double>(kPartialElems);
    L.red = c.take<double>(kRedStride);
}

int32_t read_red(const double *red, double (&h)[kRedStride], hipStream_t s) {
    CSD_HIP(hipMemcpyAsync(h, red, sizeof(h), hipMemcpyDeviceToHost, s));
    CSD_HIP(hipStreamSynchronize(s));
    return CSDYN_OK;
}

}  // namespace
}  // namespace csd

using namespace csd;

extern "C" int32_t csdyn_guess_workspace_bytes(const csdyn_opctx *ctx, size_t *bytes) {
    clear_error();
    if (!ctx || !bytes) { set_error("guess: null argument"); return CSDYN_EINVAL; }
    Carver c(nullptr);
    GuessLayout L;
    guess_layout(c, 24 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr, L);
    *bytes = c.off + 256;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_guess(csdyn_net *net, const csdyn_opctx *ctx, const double *b, const double *x1,
                               const double *x2, int32_t mode, double *guess, void *ws, size_t ws_bytes,
                               void *stream, csdyn_guess_info *info) {
    clear_error();
    if (!ctx || !x1 || !x2 || !guess) { set_error("guess: null argument"); return CSDYN_EINVAL; }
    if (mode < 0 || mode > 2) { set_error("guess: mode must be 0, 1 or 2"); return CSDYN_EINVAL; }
    if (mode > 0 && (!net || !b || !ws)) { set_error("guess: modes 1 and 2 need the network, b and a workspace"); return CSDYN_EINVAL; }
    const int64_t n = 24 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr, ncell = n / 4;
    hipStream_t s = (hipStream_t)stream;
    if (info) *info = csdyn_guess_info{-1.0, -1.0, -1.0, 0.0};
    if (mode == 0) {
        hipLaunchKernelGGL(k_extrapolate, grid_of(n), dim3(256), 0, s, x1, x2, guess, n);
        CSD_HIP(hipGetLastError());
        return CSDYN_OK;
    }
    Carver c(ws);
    GuessLayout L;
    guess_layout(c, n, L);
    if (c.off + 256 > ws_bytes) { set_error("guess: workspace %zu < %zu bytes", ws_bytes, c.off + 256); return CSDYN_ENOMEM; }
    double *Ad = L.ad_re, *re = L.ad_re + n;
    double h[kRedStride];
    // b with the VP pressure part projected, as the solve uses it
    CSD_TRY(Vec<double>::copy(L.bp, b, n, s));
    if (ctx->op.kind == CSDYN_VP) {
        CSD_TRY(Vec<double>::pmoments(L.bp, ctx->dg.vol, ncell, L.partial, L.red, s));
        CSD_TRY(read_red(L.red, h, s));
        CSD_TRY(Vec<double>::padd(L.bp, ncell, -h[0] / h[1], s));
    }
    hipLaunchKernelGGL(k_extrapolate, grid_of(n), dim3(256), 0, s, x1, x2, L.xe, n);
    CSD_HIP(hipGetLastError());
    CSD_TRY(csdyn_net_predict(net, x1, x2, guess, stream));            // x_n
    CSD_TRY(Vec<double>::copy(L.d, guess, n, s));
    CSD_TRY(Vec<double>::axpby(-1.0, L.xe, 1.0, L.d, n, s));           // d = x_n - x_e
    CSD_TRY(op_launch(ctx, L.xe, Ad, s));
    CSD_TRY(Vec<double>::copy(re, L.bp, n, s));
    CSD_TRY(Vec<double>::axpby(-1.0, Ad, 1.0, re, n, s));             // r_e = b - A x_e
    CSD_TRY(op_launch(ctx, L.d, Ad, s));                               // A d
    CSD_TRY(Vec<double>::mdot(L.ad_re, n, 2, re, L.partial, L.red, s));
    CSD_TRY(read_red(L.red, h, s));
    const double ea = h[0], ee = h[1];
    CSD_TRY(Vec<double>::mdot(Ad, n, 0, Ad, L.partial, L.red, s));
    CSD_TRY(read_red(L.red, h, s));
    const double aa = h[kRedStride - 1];
    const double res_e = std::sqrt(ee), res_n = std::sqrt(std::fmax(ee - 2.0 * ea + aa, 0.0));
    double alpha, res_g;
    if (mode == 1) {
        alpha = res_n < res_e ? 1.0 : 0.0;
        res_g = res_n < res_e ? res_n : res_e;
        if (alpha == 0.0) CSD_TRY(Vec<double>::copy(guess, L.xe, n, s));
    } else {
        alpha = aa > 0.0 ? ea / aa : 0.0;
        res_g = std::sqrt(std::fmax(ee - alpha * ea, 0.0));
        CSD_TRY(Vec<double>::copy(guess, L.xe, n, s));
        CSD_TRY(Vec<double>::axpby(alpha, L.d, 1.0, guess, n, s));     // x_e + alpha d
    }
    if (info) *info = csdyn_guess_info{res_e, res_n, res_g, alpha};
    return CSDYN_OK;
}

extern "C" int32_t csdyn_march_rhs(const csdyn_opctx *ctx, const double *v, const double *f, double dt, double *b,
                                   void *stream) {
    clear_error();
    if (!ctx || !v || !f || !b) { set_error("march_rhs: null argument"); return CSDYN_EINVAL; }
    const int64_t ncell = 6 * int64_t(ctx->g.n) * ctx->g.n * ctx->g.nr;
    hipLaunchKernelGGL(k_march_rhs, grid_of(4 * ncell), dim3(256), 0, (hipStream_t)stream, v, f, dt, b, ncell);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}
