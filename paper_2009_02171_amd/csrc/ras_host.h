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

// One triangular factor (L strictly lower, or U upper with 1/diag split off)
// of all subdomains, in the slice layout the sweep kernel reads: the rows of
// one level are grouped in slices of 64 lanes; entry q of lane l of slice s
// is at off[s] + q*64 + l.
struct SweepPack {
    std::vector<int32_t> lev_slice;  // [nlev_total + 1] first slice of each level
    std::vector<int64_t> sl_off;     // [nslice]
    std::vector<int32_t> sl_w;       // [nslice] entries per lane
    std::vector<int32_t> sl_rows;    // [nslice * 64] local row, -1 = padding lane
    std::vector<double> sl_diag;     // [nslice * 64] u_ii (U only; 0 on padding lanes)
    std::vector<double> val;         // [entries]
    std::vector<int32_t> col;        // [entries] local row index
};

struct SdInfo {
    int64_t cell_off;  // into gcell
    int64_t t_off;     // into the local-vector scratch (in components)
    int32_t nloc, own_off, nown;
    int32_t levL0, levL1, levU0, levU1;
    int32_t pad;
};

struct HostRas {
    int nsd = 0;
    int nb[3] = {0, 0, 0};
    std::vector<SdInfo> sd;
    std::vector<int32_t> gcell;  // local cell -> global cell
    std::vector<int32_t> own;    // owned local cells (indices relative to the subdomain)
    SweepPack L, U;
    int64_t tlen = 0;            // total local-vector length (components)
    int64_t nnz = 0;             // factor entries before padding
    int max_levels = 0;
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
