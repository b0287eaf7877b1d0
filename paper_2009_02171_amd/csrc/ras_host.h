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
// ordered by level; within a level they form slices of 64 lanes.  A slice
// holds floor(64 / s) rows, each on s adjacent lanes (s = ceil(width / 8) for
// the slice's widest row; lane j of a row takes entries [j * w, (j + 1) * w)
// with w = ceil(width / s)), so a lane holds at most eight entries.  A lane's entries are stored in pairs
// (values) and as one group of eight (addresses), lanes side by side, so
// that one 16-byte load per lane fetches a pair of values (FP64) or all eight
// addresses: entry e of lane l of slice s has value
// val[2 * (sl_off[s] + (e / 2) * 64 + l) + e % 2] and address
// addr[8 * (64 * s + l) + e].  Entries past a lane's part of its row have
// value 0.  A dependency is addressed by its ring slot: rows only depend on
// rows of the previous ring_depth - 1 levels, so the sweep keeps the results
// of the last ring_depth levels in a ring of ring_depth x ring_width values,
// slot = (level mod ring_depth) * ring_width + position of the row in its
// level; the rows of a slice have consecutive positions from sl_slot[s].
struct SweepPack {
    std::vector<int32_t> lev_slice;  // [nlev_total + 1] first slice of each level
    std::vector<int32_t> sl_info;    // [nslice] rows << 10 | (s - 1) << 4 | entries per lane
    std::vector<int64_t> sl_off;     // [nslice] first value pair
    std::vector<int32_t> sl_slot;    // [nslice] ring slot of the first row
    // Per lane (at the row's first lane) or per row (at slice*64 + the row's
    // index in the slice, entries past the slice's rows -1 or 0):
    std::vector<int32_t> lane_io;    // [nslice*64] L: x index; U: y index of an owned row, else -1; per row in the
                                     // ring, per lane in the box vector (not used by its sweep)
    std::vector<int32_t> lane_next;  // [nslice*64] ring: L only, per row, the row's U-sweep record (U slice*64 +
                                     // the row's index in it); box vector: the row's position in the box vector,
                                     // L per lane, U per row
    std::vector<double> lane_diag;   // [nslice*64] U only: u_ii per row
    std::vector<double> val;         // per slice: [w / 2][64] value pairs, then for an odd width w [64]
                                     // single values (the lanes' last entries); offsets in pairs
    std::vector<uint16_t> addr;      // ring slot of the dependency: per subdomain a block of
                                     // [8 * 64 * nsl] from slice SdInfo::asl*0; identical blocks stored once
    std::vector<int32_t> meta;       // [nsd][meta words] LDS metadata image of each subdomain's sweep
};

struct SdInfo {
    int32_t levL0, levL1, levU0, levU1;  // level ranges of the two sweeps
    int32_t nloc, nown;
    int32_t nrows;                   // rows of the box (4 per cell)
    int32_t slL0, nslL, slU0, nslU;  // first slice and number of slices of each sweep
    int32_t aslL0, aslU0;            // first slice of the subdomain's block in each sweep's (shared) addresses
    int64_t g0;                      // box vector: first entry of the subdomain's gather list
    int64_t offL0, offU0;            // first value pair of each sweep
    // Folded box vector (HostRas::folded): positions p >= fold share slot
    // p - fold with the first nrows - fold positions; the late positions'
    // inputs are written after the L sweep's level fold_lev, the early
    // positions' L results after the U sweep's level fold_levU (fold = nrows,
    // fold_lev = fold_levU = -1: nothing folded)
    int32_t fold, fold_lev, fold_levU;
    // box vector: the owned rows' {position, y index} pairs from own0 (4 nown
    // of them), the own_late ones first: rows whose slot is reused by the
    // fold (written out before that, at the U sweep's level fold_levU), then
    // the rest (written after the U sweep)
    int64_t own0;
    int32_t own_late;
};

// Bytes of one sweep's slice metadata as the sweep kernel keeps it in LDS
// (and as the per-subdomain images are laid out): the first slice of each
// level (relative), then per slice its first value pair (relative to the
// subdomain's first), level << 17 | slice info, and ring slot or position;
// each part 16-byte aligned.
constexpr size_t meta_bytes_for(int nsl, int nlev) {
    return ((size_t(nlev) + 1) * 4 + 15) / 16 * 16 + (size_t(nsl) * 12 + 15) / 16 * 16;
}

constexpr int64_t kBoxVectorBytes = 90 * 1024;
constexpr int kXcds = 8;  // L2 domains of the GPU; consecutive workgroups go to consecutive domains
// LDS of one workgroup of the folded FP64 box-vector sweep (metadata and
// slots): two such workgroups fit the 160 KiB of a compute unit with room for
// the allocation granularity.
constexpr int64_t kFoldBytes = 80 * 1024 - 512;
// The same for a subdomain vector above kBoxVectorBytes: one workgroup per
// compute unit, folded into the LDS one workgroup can have.
constexpr int64_t kLdsFoldBytes = 160 * 1024 - 512;
// Late inputs of a folded box vector held per thread from the gather to
// their write.
constexpr int kFoldRegs = 3;

// Workgroup size of a sweep whose widest level has `width` lanes (rounded to
// 64): one wavefront per slice of that level, at least 256 threads.
inline int sweep_threads(int width) { return width <= 256 ? 256 : (width <= 512 ? 512 : 1024); }

struct HostRas {
    int nsd = 0;
    int nb[3] = {0, 0, 0};
    std::vector<SdInfo> sd;
    SweepPack L, U;
    int ring_depth = 0, ring_width = 0;  // levels kept, lanes per level
    // Box-vector addressing: when a subdomain's whole FP64 vector fits the
    // budget below, the sweep keeps it in LDS (the gathered input, then the L
    // results, then the U results, in place) and addresses dependencies by the
    // row's position in the L sweep's order instead of a ring slot.
    bool box_vector = false;
    int box_rows = 0;  // rows of the largest subdomain
    // box vector: for each subdomain (from SdInfo::g0, SdInfo::nrows entries)
    // the x index of the row at each position, so the gather is one pass
    std::vector<int32_t> gio;
    // box vector: per subdomain (from SdInfo::own0) the owned rows' {position,
    // y index} pairs, the sweep's restricted scatter from LDS
    std::vector<int32_t> own;
    int max_slices = 0, max_levels = 0;  // per sweep of one subdomain (LDS metadata sizing)
    int64_t nnz = 0;                     // factor entries (L and U, diagonal included)
    int64_t box_cells = 0, owned_cells = 0;
    int max_total_levels = 0;            // L + U levels of the deepest subdomain
    // Workgroup b of a sweep launch solves subdomain perm[b].  Subdomains that
    // share their address blocks are dealt to the same of the kXcds L2 domains
    // (workgroup b runs on domain b mod kXcds), so each domain's L2 holds the
    // addresses of a few structures, read from HBM once.
    std::vector<int32_t> perm;
    int addr_classes = 0;                // distinct (L, U) address structures
    int meta_words = 0;                  // int32 words of one metadata image (meta_bytes_for / 4)
    // Folded box vector, for FP64 sweeps whose whole vector would keep one
    // workgroup per compute unit.  Every row keeps its position in the L
    // sweep's order; position p of a subdomain with fold point f (SdInfo::fold)
    // is stored in slot p - f when p >= f ("late"), else in slot p, so the late
    // rows reuse the slots of the first e = nrows - f rows ("early").  Valid
    // when every L-sweep access of an early row precedes the late rows' first
    // level by two levels (the late inputs, held in registers since the
    // gather, swap places with the early rows' L results in between, after
    // the level SdInfo::fold_lev), and every U-sweep access of a late row
    // precedes the early rows' first U level by two levels (the owned late
    // rows are written to y and the early rows' L results go back to their
    // slots in between, after the level SdInfo::fold_levU).  The arrays
    // below replace, for the FP64 sweep, L.addr, U.addr, L.meta and U's
    // positions (same layouts); fold_early is the largest e.
    bool folded = false;
    int fold_rows = 0, fold_early = 0;  // slots of the largest folded subdomain, its early rows
    std::vector<uint16_t> fold_Laddr, fold_Uaddr;
    std::vector<int32_t> fold_Lmeta, fold_Upos;
};

// Build and factor.  Returns CSDYN_EZEROPIVOT / CSDYN_EINVAL on failure.
// storage: 0 automatic (box vector when its FP64 size fits kBoxVectorBytes,
// folded when metadata and vector exceed kFoldBytes and the fold is valid;
// a larger box vector folded into kLdsFoldBytes when that fold is valid for
// every subdomain, else the ring), 1 ring, 2 box vector (folded as in 0),
// 3 as 0 but never folded.
int32_t build_host_ras(const HostGeom &g, const csdyn_op &op, const int sub[3], int overlap, int storage,
                       HostRas &out);

// The factor values with every odd width's last entries padded to pairs (the
// layout the FP32 sweeps and the FP64 sweeps of few subdomains read; the other
// FP64 sweeps read the packed layout of SweepPack::val): new_off[slice] is the slice's first pair, padded_pairs()
// the pairs of the whole pack (with the same tail padding as val), and
// padded_values() writes them, converted to T, into out (padded_pairs() * 2
// entries).
std::vector<int64_t> padded_offsets(const SweepPack &P);
int64_t padded_pairs(const SweepPack &P);
template <class T>
void padded_values(const SweepPack &P, const std::vector<int64_t> &new_off, T *out);
// The subdomain table and metadata images for the padded layout (each
// subdomain's first pair and its slices' relative offsets), from the L
// sweep's images Lsrc (L.meta, or fold_Lmeta for a folded FP64 sweep).
void padded_meta(const HostRas &H, const std::vector<int32_t> &Lsrc, const std::vector<int64_t> &Loff,
                 const std::vector<int64_t> &Uoff, std::vector<SdInfo> &sd, std::vector<int32_t> &Lmeta,
                 std::vector<int32_t> &Umeta);

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
