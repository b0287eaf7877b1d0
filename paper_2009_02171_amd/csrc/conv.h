// Internal launchers of the convolution kernels (conv.hip), used by the
// learned-guess network (net.hip).
#pragma once

#include "common.h"

namespace csd {

struct ConvDims {
    int nb, d, h, w;  // batch (panels) and volume
    int ci, co;       // logical channels
    int ci8, co8;     // tensor channel strides (round_up(c, 8))
    int kpad;         // packed K of the forward weights: round_up(27 ci8, 32)
    int64_t nvox;     // nb d h w
};

int32_t conv_dims(const csdyn_conv_shape *s, ConvDims &a);
void conv_packed_sizes(const ConvDims &a, int64_t &wf_elems, int64_t &wb_elems);
size_t conv_bwd_weight_ws(const ConvDims &a);
int32_t conv_pack_launch(const ConvDims &a, const float *w, uint16_t *wf, uint16_t *wb, hipStream_t s);
int32_t conv_fwd_launch(const ConvDims &a, const uint16_t *x, const uint16_t *wf, const float *bias,
                        const uint16_t *res, const uint16_t *mask, int relu, uint16_t *y, float *y32, hipStream_t s,
                        const char *name);
int32_t conv_bwd_data_launch(const ConvDims &a, const uint16_t *dy, const uint16_t *wb, const uint16_t *mask,
                             uint16_t *dx, hipStream_t s);
int32_t conv_bwd_weight_launch(const ConvDims &a, const uint16_t *x, const uint16_t *dy, float *dw, float *db,
                               void *ws, size_t ws_bytes, hipStream_t s);
// dst = scale * mean of 8 children (coarse sizes given) [+ add] [zero where mask <= 0]
int32_t pool_launch(int nb, int d, int h, int w, int c8, const uint16_t *src, float scale, const uint16_t *add,
                    const uint16_t *mask, uint16_t *dst, hipStream_t s);
// dst = scale * parent (fine sizes given) [+ add] [zero where mask <= 0]
int32_t up_launch(int nb, int d, int h, int w, int c8, const uint16_t *src, float scale, const uint16_t *add,
                  const uint16_t *mask, uint16_t *dst, hipStream_t s);
int32_t adam_launch(float *p, const float *g, float *m, float *v, int64_t n, int32_t step, float lr, float b1,
                    float b2, float eps, hipStream_t s);

}  // namespace csd
