// Host-side construction of the RAS preconditioner data (Sec. 3.3):
// subdomain boxes, the restricted matrices A_i = R_i A R_i^T with the
// structural stencil pattern, their ILU(0) factors, and the level schedule
// of the triangular sweeps packed into 64-row slices for the GPU.
#pragma once

#include <cstdint>
#include <memory>
#include <vector>

#include "common.h"

namespace csd {

// One triangular sweep (the L sweep or the U sweep) of all subdomains, in
// the order the sweep kernel processes it.  The rows of a subdomain are
// ordered by level; within a level they form slices of 64 lanes (one row per
// lane).  Entry q of lane l of slice s is at sl_off[s] + q*64 + l.  A
// dependency is addressed by its ring slot: rows only depend on rows of the
// previous ring_depth - 1 levels, so the sweep keeps the results of the last
// ring_depth levels in a ring of ring_depth x ring_width values, slot =
// (level mod ring_depth) * ring_width + 64 * (slice - first slice of the
// level) + lane.
struct SweepPack {
    std::vector<int32_t> lev_slice;  // [nlev_total + 1] first slice of each level
    std::vector<int32_t> sl_w;       // [nslice] entries per lane
    std::vector<int64_t> sl_off;     // [nslice]
    std::vector<int32_t> lane_io;    // [nslice*64] L: x index of the row; U: y index of an owned row; else -1
    std::vector<int32_t> lane_next;  // [nslice*64] L only: U-sweep position (slice*64 + lane) of the row
    std::vector<double> lane_diag;   // [nslice*64] U only: u_ii (0 on padding lanes)
    std::vector<double> val;         // [entries]
    std::vector<uint16_t> addr;      // [entries] ring slot of the dependency
};

struct SdInfo {
    int32_t levL0, levL1, levU0, levU1;  // level ranges of the two sweeps
    int32_t nloc, nown;
};

struct HostRas {
    int nsd = 0;
    int nb[3] = {0, 0, 0};
    std::vector<SdInfo> sd;
    SweepPack L, U;
    int ring_depth = 0, ring_width = 0;  // levels kept, lanes per level
    int max_slices = 0, max_levels = 0;  // per sweep of one subdomain (LDS metadata sizing)
    int64_t nnz = 0;                     // factor entries (L and U, diagonal included)
    int64_t box_cells = 0, owned_cells = 0;
    int max_total_levels = 0;            // L + U levels of the deepest subdomain
};

// Build and factor.  Returns CSDYN_EZEROPIVOT / CSDYN_EINVAL on failure.
int32_t build_host_ras(const HostGeom &g, const csdyn_op &op, const int sub[3], int overlap, HostRas &out);

// One subdomain's box cells, owned cells and ILU(0) factors as CSR (L strictly
// lower with unit diagonal implied, U upper), for inspection.
int32_t host_subdomain(const HostGeom &g, const csdyn_op &op, const int sub[3], int overlap, int s,
                       std::vector<int32_t> &gcell, std::vector<int32_t> &own, std::vector<int64_t> &rp,
                       std::vector<int32_t> &ci, std::vector<double> &v);

// Row-by-row structural expansion of A (used by the builder; exposed for
// the inspection entry point).
void stencil_row(const HostGeom &g, const csdyn_op &op, int p, int i, int j, int k, int c,
                 std::vector<std::pair<int64_t, double>> &out);

}  // namespace csd
