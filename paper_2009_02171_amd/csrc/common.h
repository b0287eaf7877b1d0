// Internal declarations shared by the libcsdyn translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>
#include <vector>

#include "../../include/csdyn.h"

namespace csd {

// ------------------------------------------------------------------ errors
void set_error(const char *fmt, ...);
void clear_error();

#define CSD_HIP(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess) {                                                                \
            ::csd::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                             __LINE__);                                                        \
            return CSDYN_EHIP;                                                                 \
        }                                                                                      \
    } while (0)

#define CSD_TRY(expr)                      \
    do {                                   \
        int32_t rc_ = (expr);              \
        if (rc_ != CSDYN_OK) return rc_;   \
    } while (0)

// Bump allocator over a caller-owned device workspace (sizes are first
// measured with a null base, then carved for real).
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// --------------------------------------------------------------- geometry
// Panel p maps local (1, tan xi, tan eta) to global Cartesian by ROT[p].
extern const int ROT[6][3][3];

struct GhostEntry {  // ghost cell beyond panel edge e at tangential index t
    int q;           // neighbour panel
    int fix_i;       // 1: neighbour line has fixed i = idx and varying j
    int idx;         // 0 or N-1
    int m0;          // first of the 4 interpolation nodes
    double w[4];     // cubic Lagrange weights in the neighbour's angle
};

struct FaceEntry {   // the same edge face seen from the neighbour panel
    int q, e, t;
};

struct HostGeom {
    int n = 0, nr = 0;
    double ri = 0, ro = 0, hs = 0, hr = 0;
    std::vector<GhostEntry> ghost;  // [6][4][n]
    std::vector<FaceEntry> face;    // [6][4][n]
    // metric tables, same layout as DevGeom
    std::vector<double> a11x, a12x, a22y, a12y, sc, t1, t2, nrm, gc1, gc2, rk, rf, vol;
    // lay[k]: r_k, 1/r_k^2, r_{k-1/2}^2, r_{k+1/2}^2, 1/(r_k h_r)^2, 1/(2 r_k^2 h_r), 1/r_k, 0
    std::vector<double> lay, isc;
    int32_t build(const csdyn_grid &g);
    size_t nf() const { return size_t(n) * (n + 1); }
    double ang(double i) const { return -0.78539816339744830962 + (i + 0.5) * hs; }
    double rad(double k) const { return ri + (k + 0.5) * hr; }
    int64_t cell(int p, int i, int j, int k) const { return ((int64_t(p) * nr + k) * n + j) * n + i; }
};

// Device-side geometry and edge buffers of one grid (pointers into the
// operator workspace).
struct DevGeom {
    int n, nr;
    double hs, hr;
    double *a11x, *a12x;  // [n][n+1]   xi-faces (row j, face index fi = 0..n)
    double *a22y, *a12y;  // [n+1][n]   eta-faces (face index fj, column i)
    double *sc;           // [n][n]     sqrt(g)/r^2 at cell centres
    double *t1;           // [6][n][n+1][3]  sqrt(g) g^1 / r at xi-faces, global frame
    double *t2;           // [6][n+1][n][3]  sqrt(g) g^2 / r at eta-faces
    double *nrm;          // [6][n][n][3]    unit radial at cell centres
    double *gc1, *gc2;    // [6][n][n][3]    r g^1, r g^2 at cell centres (dual basis, global frame)
    double *rk;           // [nr]     r_k
    double *rf;           // [nr+1]   r_{k-1/2}
    double *lay;          // [nr][8]  per-layer stencil factors (see HostGeom::lay)
    double *isc;          // [n][n]   1 / (h_s sqrt(g)/r^2) at cell centres
    double wq2_bot, wq2_top;  // (r_in / r_ghost)^2 at the inner and outer wall
    double *zero;         // [64] zeros: the source of loads that must read 0
    double *sink;         // [2048] written by threads whose result is discarded
    int *gh_i;            // [6][4][n][4]  q, fix_i, idx, m0
    double *gh_w;         // [6][4][n][4]
    int *fc;              // [6][4][n][4]  q, e, t, pad
    double *vol;          // [6][nr][n][n] cell volumes (for the Neumann projection)
    double *G;            // [6][4][nr][n][4] ghost values
    double *SF;           // averaged edge fluxes: [6][4][nr][n][4] Laplacian, then [6][4][nr][n padded to 4] divergence
};

size_t devgeom_bytes(int n, int nr);
int32_t devgeom_setup(const HostGeom &hg, void *ws, DevGeom *out);

}  // namespace csd

struct csdyn_opctx {
    csdyn_grid g;
    csdyn_op op;
    csd::HostGeom hg;
    csd::DevGeom dg;
    void *ws;
    size_t ws_bytes;
    int32_t tile = 0;  // stencil workgroup shape: 0 default (16x8), 1: 32x8, 2: 16x16, 3: 64x4, 4: 16x8, 5: 32x4
};

namespace csd {
// Preconditioner apply (FP64 in and out) and its properties (ras.hip).
int32_t ras_apply_d(const csdyn_ras *pc, const double *x, double *y, hipStream_t s);
int ras_levels(const csdyn_ras *pc);
const csdyn_opctx *ras_fine_ctx(const csdyn_ras *pc);
// Launch the three operator kernels (ghost fill, edge fluxes, stencil).
int32_t op_launch(const csdyn_opctx *ctx, const double *x, double *y, hipStream_t s);
// FP32 variant used inside the FP32 preconditioner.
int32_t op_launch_f32(const csdyn_opctx *ctx, const float *x, float *y, float *G32, float *SF32, hipStream_t s);
}  // namespace csd
