// Learned initial guess for the GMRES solves (the paper takes x0 from the
// previous time step, Sec. 3.3): a panel-wise 3-D convolutional network that
// predicts a correction to linear extrapolation from the previous two
// solutions, trained online by Adam on the solutions the solver produces.
//
// Network (channel widths c0..c3, four resolution levels, additive skips):
//   e0 = relu(conv0(x))  e1 = relu(conv1(pool e0))  e2 = relu(conv2(pool e1))
//   e3 = relu(conv3(pool e2))  d2 = relu(conv4(up e3) + e2)
//   d1 = relu(conv5(up d2) + e1)  d0 = relu(conv6(up d1) + e0)  y = conv7(d0)
// Features: x = (x1 / s, (x1 - x2) / sd) with s, sd the per-component RMS;
// guess = 2 x1 - x2 + sd * y; loss = mean (y - (xn - 2 x1 + x2) / sd)^2.
// Activations and weights BF16, accumulation and master weights FP32,
// features, scales, loss and guess FP64.
#include <cmath>
#include <cstring>
#include <memory>

#include "common.h"
#include "conv.h"
#include "profile.h"

namespace csd {

namespace {

constexpr int kMomBlocks = 512;

__device__ inline uint16_t f2bf_n(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return uint16_t(u >> 16);
}

// partial[b][0..3] = sum x1_c^2, partial[b][4..7] = sum (x1 - x2)_c^2 over the block's cells
__global__ __launch_bounds__(256) void k_moments(int64_t ncell, const double *__restrict__ x1,
                                                 const double *__restrict__ x2, double *__restrict__ partial) {
    __shared__ double red[8][256];
    double s[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int64_t per = (ncell + gridDim.x - 1) / gridDim.x;
    const int64_t c0 = int64_t(blockIdx.x) * per, c1 = c0 + per < ncell ? c0 + per : ncell;
    for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x)
        for (int q = 0; q < 4; ++q) {
            const double a = x1[4 * c + q], d = a - x2[4 * c + q];
            s[q] += a * a;
            s[4 + q] += d * d;
        }
    for (int q = 0; q < 8; ++q) red[q][threadIdx.x] = s[q];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w)
            for (int q = 0; q < 8; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 8) partial[size_t(blockIdx.x) * 8 + threadIdx.x] = red[threadIdx.x][0];
}

// scal[0..3] = s, scal[4..7] = sd (RMS + 1e-30)
__global__ void k_moments_final(int nblk, int64_t ncell, const double *__restrict__ partial, double *__restrict__ scal) {
    const int q = threadIdx.x;
    if (q >= 8) return;
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += partial[size_t(b) * 8 + q];
    scal[q] = sqrt(s / double(ncell)) + 1e-30;
}

__global__ void k_features(int64_t ncell, const double *__restrict__ x1, const double *__restrict__ x2,
                           const double *__restrict__ scal, uint16_t *__restrict__ x) {
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (c >= ncell) return;
    for (int q = 0; q < 4; ++q) {
        const double a = x1[4 * c + q], d = a - x2[4 * c + q];
        x[8 * c + q] = f2bf_n(float(a / scal[q]));
        x[8 * c + 4 + q] = f2bf_n(float(d / scal[4 + q]));
    }
}

// dy = d loss / d y (8 channels, 4..7 zero), partial loss sums per block
__global__ __launch_bounds__(256) void k_loss(int64_t ncell, const float *__restrict__ y, const double *__restrict__ xn,
                                              const double *__restrict__ x1, const double *__restrict__ x2,
                                              const double *__restrict__ scal, uint16_t *__restrict__ dy,
                                              double *__restrict__ partial) {
    __shared__ double red[256];
    const int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    double s = 0;
    if (c < ncell) {
        const double inv = 2.0 / (4.0 * double(ncell));
        for (int q = 0; q < 4; ++q) {
            const double t = (xn[4 * c + q] - 2.0 * x1[4 * c + q] + x2[4 * c + q]) / scal[4 + q];
            const double diff = double(y[4 * c + q]) - t;
            s += diff * diff;
            dy[8 * c + q] = f2bf_n(float(inv * diff));
            dy[8 * c + 4 + q] = 0;
        }
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (int(threadIdx.x) < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_loss_final(int nblk, int64_t ncell, const double *__restrict__ partial, double *__restrict__ out) {
    if (threadIdx.x != 0) return;
    double s = 0;
    for (int b = 0; b < nblk; ++b) s += partial[b];
    out[0] = s / (4.0 * double(ncell));
}

__global__ void k_guess(int64_t ncell, const float *__restrict__ y, const double *__restrict__ x1,
                        const double *__restrict__ x2, const double *__restrict__ scal, double *__restrict__ out) {
    const int64_t e = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
    if (e >= 4 * ncell) return;
    const int q = int(e & 3);
    out[e] = 2.0 * x1[e] - x2[e] + scal[4 + q] * double(y[e]);
}

inline int rup8(int c) { return (c + 7) / 8 * 8; }

}  // namespace

struct NetLayer {
    ConvDims a;
    int64_t woff, boff;  // offsets of W [co][27][ci] and b [co] in the flat parameter vector
    uint16_t *wf = nullptr, *wb = nullptr;
};

}  // namespace csd

struct csdyn_net {
    int n = 0, nr = 0, widths[4] = {0, 0, 0, 0};
    int64_t vox[4] = {0, 0, 0, 0};  // voxels per level (all six panels)
    csd::NetLayer L[8];
    int64_t nparam = 0;
    int32_t step = 0;
    float *params = nullptr, *grads = nullptr, *m = nullptr, *v = nullptr;
    uint16_t *x = nullptr, *e0 = nullptr, *p0 = nullptr, *e1 = nullptr, *p1 = nullptr, *e2 = nullptr, *p2 = nullptr,
             *e3 = nullptr, *u3 = nullptr, *d2 = nullptr, *u2 = nullptr, *d1 = nullptr, *u1 = nullptr, *d0 = nullptr;
    float *y = nullptr;
    uint16_t *dy = nullptr, *dz[7] = {}, *tmp = nullptr;
    double *scal = nullptr, *mom = nullptr, *lpart = nullptr, *loss = nullptr;
    void *bwdw = nullptr;
    size_t bwdw_bytes = 0;
};

namespace csd {

static int32_t net_check(int32_t n, int32_t nr, const int32_t *widths) {
    if (!widths) { set_error("net: null widths"); return CSDYN_EINVAL; }
    if (n < 8 || nr < 8 || n % 8 || nr % 8) {
        set_error("net: N and Nr must be multiples of 8 (four levels), got %d, %d", n, nr);
        return CSDYN_EINVAL;
    }
    for (int l = 0; l < 4; ++l)
        if (widths[l] < 1 || widths[l] > 128) { set_error("net: widths must be in [1, 128]"); return CSDYN_EINVAL; }
    return CSDYN_OK;
}

// layer l: (level, cin, cout)
static void layer_spec(const int32_t *w, int l, int &lev, int &ci, int &co) {
    const int c0 = w[0], c1 = w[1], c2 = w[2], c3 = w[3];
    const int spec[8][3] = {{0, 8, c0}, {1, c0, c1}, {2, c1, c2}, {3, c2, c3},
                            {2, c3, c2}, {1, c2, c1}, {0, c1, c0}, {0, c0, 4}};
    lev = spec[l][0];
    ci = spec[l][1];
    co = spec[l][2];
}

static int64_t param_count(const int32_t *w) {
    int64_t s = 0;
    for (int l = 0; l < 8; ++l) {
        int lev, ci, co;
        layer_spec(w, l, lev, ci, co);
        s += int64_t(co) * 27 * ci + co;
    }
    return s;
}

// Carve everything (c.base == nullptr: measure only).
static int32_t net_carve(csdyn_net *nt, Carver &c) {
    const int n = nt->n, nr = nt->nr;
    for (int lv = 0; lv < 4; ++lv) nt->vox[lv] = 6 * int64_t(nr >> lv) * (n >> lv) * (n >> lv);
    int64_t off = 0;
    for (int l = 0; l < 8; ++l) {
        int lev, ci, co;
        layer_spec(nt->widths, l, lev, ci, co);
        csdyn_conv_shape s{6, nr >> lev, n >> lev, n >> lev, ci, co};
        CSD_TRY(conv_dims(&s, nt->L[l].a));
        nt->L[l].woff = off;
        off += int64_t(co) * 27 * ci;
        nt->L[l].boff = off;
        off += co;
    }
    nt->nparam = off;
    nt->params = c.take<float>(off);
    nt->grads = c.take<float>(off);
    nt->m = c.take<float>(off);
    nt->v = c.take<float>(off);
    for (int l = 0; l < 8; ++l) {
        int64_t nf, nb;
        conv_packed_sizes(nt->L[l].a, nf, nb);
        nt->L[l].wf = c.take<uint16_t>(nf);
        nt->L[l].wb = c.take<uint16_t>(nb);
    }
    const int C0 = rup8(nt->widths[0]), C1 = rup8(nt->widths[1]), C2 = rup8(nt->widths[2]),
              C3 = rup8(nt->widths[3]);
    const int64_t *V = nt->vox;
    nt->x = c.take<uint16_t>(V[0] * 8);
    nt->e0 = c.take<uint16_t>(V[0] * C0);
    nt->p0 = c.take<uint16_t>(V[1] * C0);
    nt->e1 = c.take<uint16_t>(V[1] * C1);
    nt->p1 = c.take<uint16_t>(V[2] * C1);
    nt->e2 = c.take<uint16_t>(V[2] * C2);
    nt->p2 = c.take<uint16_t>(V[3] * C2);
    nt->e3 = c.take<uint16_t>(V[3] * C3);
    nt->u3 = c.take<uint16_t>(V[2] * C3);
    nt->d2 = c.take<uint16_t>(V[2] * C2);
    nt->u2 = c.take<uint16_t>(V[1] * C2);
    nt->d1 = c.take<uint16_t>(V[1] * C1);
    nt->u1 = c.take<uint16_t>(V[0] * C1);
    nt->d0 = c.take<uint16_t>(V[0] * C0);
    nt->y = c.take<float>(V[0] * 4);
    nt->dy = c.take<uint16_t>(V[0] * 8);
    // dz[l]: pre-activation gradient of layer l's output (l = 0..6)
    const int64_t dzs[7] = {V[0] * C0, V[1] * C1, V[2] * C2, V[3] * C3, V[2] * C2, V[1] * C1, V[0] * C0};
    for (int l = 0; l < 7; ++l) nt->dz[l] = c.take<uint16_t>(dzs[l]);
    int64_t tmax = 0;
    const int64_t tcand[6] = {V[0] * C1, V[1] * C2, V[2] * C3, V[3] * C2, V[2] * C1, V[1] * C0};
    for (int64_t t : tcand) tmax = t > tmax ? t : tmax;
    nt->tmp = c.take<uint16_t>(tmax);
    nt->scal = c.take<double>(8);
    nt->mom = c.take<double>(size_t(kMomBlocks) * 8);
    nt->lpart = c.take<double>((V[0] + 255) / 256);
    nt->loss = c.take<double>(1);
    size_t wsb = 0;
    for (int l = 0; l < 8; ++l) {
        const size_t b = conv_bwd_weight_ws(nt->L[l].a);
        wsb = b > wsb ? b : wsb;
    }
    nt->bwdw = c.take<char>(wsb);
    nt->bwdw_bytes = wsb;
    return CSDYN_OK;
}

static int32_t net_pack(csdyn_net *nt, hipStream_t s) {
    for (int l = 0; l < 8; ++l)
        CSD_TRY(conv_pack_launch(nt->L[l].a, nt->params + nt->L[l].woff, nt->L[l].wf, nt->L[l].wb, s));
    return CSDYN_OK;
}

static int32_t net_features(csdyn_net *nt, const double *x1, const double *x2, hipStream_t s) {
    const int64_t nc = nt->vox[0];
    hipLaunchKernelGGL(k_moments, dim3(kMomBlocks), dim3(256), 0, s, nc, x1, x2, nt->mom);
    hipLaunchKernelGGL(k_moments_final, dim3(1), dim3(64), 0, s, kMomBlocks, nc, nt->mom, nt->scal);
    hipLaunchKernelGGL(k_features, dim3(unsigned((nc + 255) / 256)), dim3(256), 0, s, nc, x1, x2, nt->scal, nt->x);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

static int32_t net_forward(csdyn_net *nt, hipStream_t s) {
    auto P = [&](int l, int64_t off) { return nt->params + off; };
    auto conv = [&](int l, const uint16_t *in, const uint16_t *res, uint16_t *out, float *out32, int relu) {
        const NetLayer &L = nt->L[l];
        return conv_fwd_launch(L.a, in, L.wf, P(l, L.boff), res, nullptr, relu, out, out32, s, "conv_fwd");
    };
    const int n = nt->n, nr = nt->nr;
    const int C0 = rup8(nt->widths[0]), C1 = rup8(nt->widths[1]), C2 = rup8(nt->widths[2]),
              C3 = rup8(nt->widths[3]);
    CSD_TRY(conv(0, nt->x, nullptr, nt->e0, nullptr, 1));
    CSD_TRY(pool_launch(6, nr / 2, n / 2, n / 2, C0, nt->e0, 1.f, nullptr, nullptr, nt->p0, s));
    CSD_TRY(conv(1, nt->p0, nullptr, nt->e1, nullptr, 1));
    CSD_TRY(pool_launch(6, nr / 4, n / 4, n / 4, C1, nt->e1, 1.f, nullptr, nullptr, nt->p1, s));
    CSD_TRY(conv(2, nt->p1, nullptr, nt->e2, nullptr, 1));
    CSD_TRY(pool_launch(6, nr / 8, n / 8, n / 8, C2, nt->e2, 1.f, nullptr, nullptr, nt->p2, s));
    CSD_TRY(conv(3, nt->p2, nullptr, nt->e3, nullptr, 1));
    CSD_TRY(up_launch(6, nr / 4, n / 4, n / 4, C3, nt->e3, 1.f, nullptr, nullptr, nt->u3, s));
    CSD_TRY(conv(4, nt->u3, nt->e2, nt->d2, nullptr, 1));
    CSD_TRY(up_launch(6, nr / 2, n / 2, n / 2, C2, nt->d2, 1.f, nullptr, nullptr, nt->u2, s));
    CSD_TRY(conv(5, nt->u2, nt->e1, nt->d1, nullptr, 1));
    CSD_TRY(up_launch(6, nr, n, n, C1, nt->d1, 1.f, nullptr, nullptr, nt->u1, s));
    CSD_TRY(conv(6, nt->u1, nt->e0, nt->d0, nullptr, 1));
    CSD_TRY(conv(7, nt->d0, nullptr, nullptr, nt->y, 0));
    return CSDYN_OK;
}

// Gradients of the loss into nt->grads (dy must hold d loss / d y).
static int32_t net_backward(csdyn_net *nt, hipStream_t s) {
    const int n = nt->n, nr = nt->nr;
    const int C0 = rup8(nt->widths[0]), C1 = rup8(nt->widths[1]), C2 = rup8(nt->widths[2]);
    auto G = [&](int l, const uint16_t *in, const uint16_t *dz) {
        const NetLayer &L = nt->L[l];
        return conv_bwd_weight_launch(L.a, in, dz, nt->grads + L.woff, nt->grads + L.boff, nt->bwdw, nt->bwdw_bytes,
                                      s);
    };
    auto D = [&](int l, const uint16_t *dz, const uint16_t *mask, uint16_t *out) {
        const NetLayer &L = nt->L[l];
        return conv_bwd_data_launch(L.a, dz, L.wb, mask, out, s);
    };
    uint16_t **dz = nt->dz;
    CSD_TRY(G(7, nt->d0, nt->dy));
    CSD_TRY(D(7, nt->dy, nt->d0, dz[6]));  // through relu of d0
    CSD_TRY(G(6, nt->u1, dz[6]));
    CSD_TRY(D(6, dz[6], nullptr, nt->tmp));
    CSD_TRY(pool_launch(6, nr / 2, n / 2, n / 2, C1, nt->tmp, 8.f, nullptr, nt->d1, dz[5], s));
    CSD_TRY(G(5, nt->u2, dz[5]));
    CSD_TRY(D(5, dz[5], nullptr, nt->tmp));
    CSD_TRY(pool_launch(6, nr / 4, n / 4, n / 4, C2, nt->tmp, 8.f, nullptr, nt->d2, dz[4], s));
    CSD_TRY(G(4, nt->u3, dz[4]));
    CSD_TRY(D(4, dz[4], nullptr, nt->tmp));
    CSD_TRY(pool_launch(6, nr / 8, n / 8, n / 8, rup8(nt->widths[3]), nt->tmp, 8.f, nullptr, nt->e3, dz[3], s));
    CSD_TRY(G(3, nt->p2, dz[3]));
    CSD_TRY(D(3, dz[3], nullptr, nt->tmp));
    CSD_TRY(up_launch(6, nr / 4, n / 4, n / 4, C2, nt->tmp, 0.125f, dz[4], nt->e2, dz[2], s));
    CSD_TRY(G(2, nt->p1, dz[2]));
    CSD_TRY(D(2, dz[2], nullptr, nt->tmp));
    CSD_TRY(up_launch(6, nr / 2, n / 2, n / 2, C1, nt->tmp, 0.125f, dz[5], nt->e1, dz[1], s));
    CSD_TRY(G(1, nt->p0, dz[1]));
    CSD_TRY(D(1, dz[1], nullptr, nt->tmp));
    CSD_TRY(up_launch(6, nr, n, n, C0, nt->tmp, 0.125f, dz[6], nt->e0, dz[0], s));
    CSD_TRY(G(0, nt->x, dz[0]));
    return CSDYN_OK;
}

static int32_t net_loss(csdyn_net *nt, const double *xn, const double *x1, const double *x2, hipStream_t s) {
    const int64_t nc = nt->vox[0];
    const int nblk = int((nc + 255) / 256);
    hipLaunchKernelGGL(k_loss, dim3(nblk), dim3(256), 0, s, nc, nt->y, xn, x1, x2, nt->scal, nt->dy, nt->lpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, nblk, nc, nt->lpart, nt->loss);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

static int32_t read_loss(csdyn_net *nt, double *loss, hipStream_t s) {
    if (!loss) return CSDYN_OK;
    CSD_HIP(hipMemcpyAsync(loss, nt->loss, sizeof(double), hipMemcpyDeviceToHost, s));
    CSD_HIP(hipStreamSynchronize(s));
    return CSDYN_OK;
}

}  // namespace csd

using namespace csd;

extern "C" int32_t csdyn_net_param_count(const int32_t *widths, int64_t *count) {
    clear_error();
    if (!widths || !count) { set_error("csdyn_net_param_count: null pointer"); return CSDYN_EINVAL; }
    *count = param_count(widths);
    return CSDYN_OK;
}

extern "C" int32_t csdyn_net_workspace_bytes(int32_t n, int32_t nr, const int32_t *widths, size_t *bytes) {
    clear_error();
    CSD_TRY(net_check(n, nr, widths));
    if (!bytes) { set_error("csdyn_net_workspace_bytes: null pointer"); return CSDYN_EINVAL; }
    csdyn_net tmp;
    tmp.n = n;
    tmp.nr = nr;
    std::memcpy(tmp.widths, widths, sizeof(tmp.widths));
    Carver c(nullptr);
    CSD_TRY(net_carve(&tmp, c));
    *bytes = c.off + 256;
    return CSDYN_OK;
}

extern "C" int32_t csdyn_net_setup(int32_t n, int32_t nr, const int32_t *widths, const float *params, void *ws,
                                   size_t ws_bytes, void *stream, csdyn_net **out) {
    clear_error();
    CSD_TRY(net_check(n, nr, widths));
    if (!params || !ws || !out) { set_error("csdyn_net_setup: null pointer"); return CSDYN_EINVAL; }
    size_t need = 0;
    CSD_TRY(csdyn_net_workspace_bytes(n, nr, widths, &need));
    if (ws_bytes < need) { set_error("csdyn_net_setup: workspace %zu < %zu bytes", ws_bytes, need); return CSDYN_ENOMEM; }
    std::unique_ptr<csdyn_net> nt(new csdyn_net);
    nt->n = n;
    nt->nr = nr;
    std::memcpy(nt->widths, widths, sizeof(nt->widths));
    Carver c(ws);
    CSD_TRY(net_carve(nt.get(), c));
    hipStream_t s = (hipStream_t)stream;
    CSD_HIP(hipMemcpyAsync(nt->params, params, nt->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
    CSD_HIP(hipMemsetAsync(nt->m, 0, nt->nparam * sizeof(float), s));
    CSD_HIP(hipMemsetAsync(nt->v, 0, nt->nparam * sizeof(float), s));
    CSD_TRY(net_pack(nt.get(), s));
    *out = nt.release();
    return CSDYN_OK;
}

extern "C" int32_t csdyn_net_get_params(const csdyn_net *nt, float *params, void *stream) {
    clear_error();
    if (!nt || !params) { set_error("csdyn_net_get_params: null pointer"); return CSDYN_EINVAL; }
    CSD_HIP(hipMemcpyAsync(params, nt->params, nt->nparam * sizeof(float), hipMemcpyDeviceToDevice,
                           (hipStream_t)stream));
    return CSDYN_OK;
}

extern "C" int32_t csdyn_net_predict(csdyn_net *nt, const double *x1, const double *x2, double *guess,
                                     void *stream) {
    clear_error();
    if (!nt || !x1 || !x2 || !guess) { set_error("csdyn_net_predict: null pointer"); return CSDYN_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    CSD_TRY(net_features(nt, x1, x2, s));
    CSD_TRY(net_forward(nt, s));
    const int64_t ne = 4 * nt->vox[0];
    hipLaunchKernelGGL(k_guess, dim3(unsigned((ne + 255) / 256)), dim3(256), 0, s, nt->vox[0], nt->y, x1, x2,
                       nt->scal, guess);
    CSD_HIP(hipGetLastError());
    return CSDYN_OK;
}

extern "C" int32_t csdyn_net_loss_grad(csdyn_net *nt, const double *x2, const double *x1, const double *xn,
                                       float *grads, double *loss, void *stream) {
    clear_error();
    if (!nt || !x1 || !x2 || !xn) { set_error("csdyn_net_loss_grad: null pointer"); return CSDYN_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    CSD_TRY(net_features(nt, x1, x2, s));
    CSD_TRY(net_forward(nt, s));
    CSD_TRY(net_loss(nt, xn, x1, x2, s));
    CSD_TRY(net_backward(nt, s));
    if (grads)
        CSD_HIP(hipMemcpyAsync(grads, nt->grads, nt->nparam * sizeof(float), hipMemcpyDeviceToDevice, s));
    return read_loss(nt, loss, s);
}

extern "C" int32_t csdyn_net_train_step(csdyn_net *nt, const double *x2, const double *x1, const double *xn,
                                        float lr, double *loss, void *stream) {
    clear_error();
    if (!nt || !x1 || !x2 || !xn || !(lr >= 0.f)) { set_error("csdyn_net_train_step: bad argument"); return CSDYN_EINVAL; }
    hipStream_t s = (hipStream_t)stream;
    CSD_TRY(net_features(nt, x1, x2, s));
    CSD_TRY(net_forward(nt, s));
    CSD_TRY(net_loss(nt, xn, x1, x2, s));
    CSD_TRY(net_backward(nt, s));
    nt->step += 1;
    CSD_TRY(adam_launch(nt->params, nt->grads, nt->m, nt->v, nt->nparam, nt->step, lr, 0.9f, 0.999f, 1e-8f, s));
    CSD_TRY(net_pack(nt, s));
    return read_loss(nt, loss, s);
}

extern "C" void csdyn_net_destroy(csdyn_net *nt) { delete nt; }
