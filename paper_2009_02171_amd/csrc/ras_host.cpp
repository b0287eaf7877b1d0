// Host construction of the RAS / ILU(0) data (Sec. 3.3, eq. onelevel).
#include "ras_host.h"

#include <omp.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <numeric>
#include <string>

namespace csd {

namespace {

using TermVec = std::vector<std::pair<int64_t, double>>;

// Structural expansion of one row of A into (global unknown, weight) terms.
// Every term of the stencil formula is emitted whatever its value, so the
// set of columns is the structural pattern.
class Expander {
   public:
    Expander(const HostGeom &g, const csdyn_op &op, TermVec &out) : g_(g), op_(op), out_(out) {}

    // value of component c at extended position (p, i, j, k)
    void value(int p, int i, int j, int k, int c, double w) {
        const int n = g_.n, nr = g_.nr;
        if (k < 0 || k >= nr) {
            const int kin = k < 0 ? 0 : nr - 1;
            if (op_.kind == CSDYN_VP) {
                value(p, i, j, kin, c, c < 3 ? -w : w);
            } else if (op_.kind == CSDYN_VT) {  // no-slip u, isothermal Theta
                value(p, i, j, kin, c, -w);
            } else if (c == 3) {
                value(p, i, j, kin, 3, -w);
            } else {
                const double rg = k < 0 ? g_.rf[0] - 0.5 * g_.hr : g_.rf[nr] + 0.5 * g_.hr;
                const double q = (g_.rk[kin] / rg) * (g_.rk[kin] / rg);
                const double *nv = &g_.nrm[((size_t(p) * n + j) * n + i) * 3];
                for (int d = 0; d < 3; ++d) value(p, i, j, kin, d, w * ((c == d ? -1.0 : 0.0) + (1.0 + q) * nv[c] * nv[d]));
            }
            return;
        }
        const bool iin = i >= 0 && i < n, jin = j >= 0 && j < n;
        if (iin && jin) {
            out_.emplace_back(4 * g_.cell(p, i, j, k) + c, w);
            return;
        }
        if (!iin && !jin) {
            const int ic = i < 0 ? 0 : n - 1, jc = j < 0 ? 0 : n - 1;
            value(p, i, jc, k, c, w);
            value(p, ic, j, k, c, w);
            value(p, ic, jc, k, c, -w);
            return;
        }
        const int e = !iin ? (i < 0 ? 0 : 1) : (j < 0 ? 2 : 3);
        const int t = !iin ? j : i;
        const GhostEntry &G = g_.ghost[(p * 4 + e) * size_t(n) + t];
        for (int m = 0; m < 4; ++m) {
            if (G.fix_i) value(G.q, G.idx, G.m0 + m, k, c, w * G.w[m]);
            else value(G.q, G.m0 + m, G.idx, k, c, w * G.w[m]);
        }
    }

    // one-sided outward Laplacian flux of component c through lateral face f
    // (0 W, 1 E, 2 S, 3 N) of cell (p, i, j, k), times w
    void lap_face(int p, int i, int j, int k, int f, int c, double w) {
        const int n = g_.n;
        const double ih = 1.0 / g_.hs, i4h = 0.25 / g_.hs;
        if (f <= 1) {
            const int fi = f == 0 ? i : i + 1, il = fi - 1, ir = fi;
            const size_t a = size_t(j) * (n + 1) + fi;
            const double s = f == 1 ? w : -w;
            const double a11 = g_.a11x[a] * ih * s, a12 = g_.a12x[a] * i4h * s;
            value(p, ir, j, k, c, a11);
            value(p, il, j, k, c, -a11);
            value(p, il, j + 1, k, c, a12);
            value(p, ir, j + 1, k, c, a12);
            value(p, il, j - 1, k, c, -a12);
            value(p, ir, j - 1, k, c, -a12);
        } else {
            const int fj = f == 2 ? j : j + 1, jl = fj - 1, jr = fj;
            const size_t a = size_t(fj) * n + i;
            const double s = f == 3 ? w : -w;
            const double a22 = g_.a22y[a] * ih * s, a12 = g_.a12y[a] * i4h * s;
            value(p, i, jr, k, c, a22);
            value(p, i, jl, k, c, -a22);
            value(p, i + 1, jl, k, c, a12);
            value(p, i + 1, jr, k, c, a12);
            value(p, i - 1, jl, k, c, -a12);
            value(p, i - 1, jr, k, c, -a12);
        }
    }

    // one-sided outward divergence flux (sqrt(g) g^m / r) . (v_c + v_nb)/2
    void div_face(int p, int i, int j, int k, int f, double w) {
        const int n = g_.n;
        const size_t nf = g_.nf();
        int ni = i, nj = j;
        const double *tv;
        if (f <= 1) {
            const int fi = f == 0 ? i : i + 1;
            ni = f == 0 ? i - 1 : i + 1;
            tv = &g_.t1[(p * nf + size_t(j) * (n + 1) + fi) * 3];
        } else {
            const int fj = f == 2 ? j : j + 1;
            nj = f == 2 ? j - 1 : j + 1;
            tv = &g_.t2[(p * nf + size_t(fj) * n + i) * 3];
        }
        const double s = (f == 1 || f == 3) ? 0.5 * w : -0.5 * w;
        for (int d = 0; d < 3; ++d) {
            value(p, i, j, k, d, s * tv[d]);
            value(p, ni, nj, k, d, s * tv[d]);
        }
    }

    bool on_edge(int i, int j, int f) const {
        return (f == 0 && i == 0) || (f == 1 && i == g_.n - 1) || (f == 2 && j == 0) || (f == 3 && j == g_.n - 1);
    }

    // cell of the neighbour panel across edge face f of (i, j)
    void partner(int p, int i, int j, int f, int &q, int &iq, int &jq, int &fq) const {
        const FaceEntry &F = g_.face[(p * 4 + f) * size_t(g_.n) + (f <= 1 ? j : i)];
        q = F.q; fq = F.e;
        switch (F.e) {
            case 0: iq = 0; jq = F.t; break;
            case 1: iq = g_.n - 1; jq = F.t; break;
            case 2: iq = F.t; jq = 0; break;
            default: iq = F.t; jq = g_.n - 1; break;
        }
    }

    // w * lap(component c) at cell (p, i, j, k)
    void laplacian(int p, int i, int j, int k, int c, double w) {
        const int n = g_.n;
        const double rk = g_.rk[k];
        const double wl = w / (rk * rk * g_.sc[size_t(j) * n + i] * g_.hs);
        for (int f = 0; f < 4; ++f) {
            if (!on_edge(i, j, f)) { lap_face(p, i, j, k, f, c, wl); continue; }
            int q, iq, jq, fq;
            partner(p, i, j, f, q, iq, jq, fq);
            lap_face(p, i, j, k, f, c, 0.5 * wl);
            lap_face(q, iq, jq, k, fq, c, -0.5 * wl);
        }
        const double wr = w / (rk * rk * g_.hr * g_.hr);
        const double up = g_.rf[k + 1] * g_.rf[k + 1] * wr, dn = g_.rf[k] * g_.rf[k] * wr;
        value(p, i, j, k + 1, c, up);
        value(p, i, j, k, c, -up);
        value(p, i, j, k, c, -dn);
        value(p, i, j, k - 1, c, dn);
    }

    // w * D(v) at cell (p, i, j, k), v = components 0..2
    void divergence(int p, int i, int j, int k, double w) {
        const int n = g_.n;
        const double rk = g_.rk[k];
        const double wl = w / (rk * g_.sc[size_t(j) * n + i] * g_.hs);
        for (int f = 0; f < 4; ++f) {
            if (!on_edge(i, j, f)) { div_face(p, i, j, k, f, wl); continue; }
            int q, iq, jq, fq;
            partner(p, i, j, f, q, iq, jq, fq);
            div_face(p, i, j, k, f, 0.5 * wl);
            div_face(q, iq, jq, k, fq, -0.5 * wl);
        }
        const double wr = 0.5 * w / (rk * rk * g_.hr);
        const double up = g_.rf[k + 1] * g_.rf[k + 1] * wr, dn = g_.rf[k] * g_.rf[k] * wr;
        const double *nv = &g_.nrm[((size_t(p) * n + j) * n + i) * 3];
        for (int d = 0; d < 3; ++d) {
            value(p, i, j, k, d, up * nv[d]);
            value(p, i, j, k + 1, d, up * nv[d]);
            value(p, i, j, k - 1, d, -dn * nv[d]);
            value(p, i, j, k, d, -dn * nv[d]);
        }
    }

    void row(int p, int i, int j, int k, int c) {
        const double dt = op_.dt, E = op_.ekman;
        if (op_.kind == CSDYN_VT) {  // velocity-temperature rows (pointwise couplings at the cell centre)
            const double *nv = &g_.nrm[((size_t(p) * g_.n + j) * g_.n + i) * 3];
            const double r = g_.rk[k];
            if (c == 3) {
                value(p, i, j, k, 3, 1.0);
                laplacian(p, i, j, k, 3, -dt * E / op_.pr);
                for (int d = 0; d < 3; ++d) value(p, i, j, k, d, -dt * E * g_.ri * g_.ro / (r * r) * nv[d]);
                return;
            }
            value(p, i, j, k, c, 1.0);
            laplacian(p, i, j, k, c, -dt * E);
            if (c == 0) value(p, i, j, k, 1, -2.0 * dt);
            if (c == 1) value(p, i, j, k, 0, 2.0 * dt);
            value(p, i, j, k, 3, -dt * op_.ra / g_.ro * r * nv[c]);
            return;
        }
        if (c == 3) {
            divergence(p, i, j, k, 1.0);
            laplacian(p, i, j, k, 3, -dt);
            return;
        }
        value(p, i, j, k, c, 1.0);
        if (op_.kind == CSDYN_VP) {
            laplacian(p, i, j, k, c, -dt * E);
            if (c == 0) value(p, i, j, k, 1, -2.0 * dt);
            if (c == 1) value(p, i, j, k, 0, 2.0 * dt);
        } else {
            laplacian(p, i, j, k, c, -dt * E / op_.pm);
        }
    }

   private:
    const HostGeom &g_;
    const csdyn_op &op_;
    TermVec &out_;
};

struct LocalSd {
    std::vector<int32_t> gcell, own;
    std::vector<uint8_t> owned_row;  // per local cell
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
    std::vector<int64_t> diag;
    std::vector<int32_t> levL, levU;  // per row
    int nlevL = 0, nlevU = 0;
    int32_t status = CSDYN_OK;
};

// Global cell reached from box position (p, i, j, k): the cell itself, the
// neighbour panel's first-layer cell across an edge face, or -1 (beyond a
// wall, or a cube-corner position).
int64_t box_cell(const HostGeom &g, int p, int i, int j, int k) {
    const int n = g.n;
    if (k < 0 || k >= g.nr) return -1;
    const bool iin = i >= 0 && i < n, jin = j >= 0 && j < n;
    if (iin && jin) return g.cell(p, i, j, k);
    if (!iin && !jin) return -1;
    if (i < -1 || i > n || j < -1 || j > n) return -1;
    const int f = !iin ? (i < 0 ? 0 : 1) : (j < 0 ? 2 : 3);
    const FaceEntry &F = g.face[(p * 4 + f) * size_t(n) + (!iin ? j : i)];
    int iq, jq;
    switch (F.e) {
        case 0: iq = 0; jq = F.t; break;
        case 1: iq = n - 1; jq = F.t; break;
        case 2: iq = F.t; jq = 0; break;
        default: iq = F.t; jq = n - 1; break;
    }
    return g.cell(F.q, iq, jq, k);
}

void build_one(const HostGeom &g, const csdyn_op &op, const int sub[3], const int nb[3], int overlap, int s,
               std::vector<int32_t> &g2l, LocalSd &L) {
    const int bi = s % nb[0], bj = (s / nb[0]) % nb[1], bk = (s / (nb[0] * nb[1])) % nb[2];
    const int p = s / (nb[0] * nb[1] * nb[2]);
    const int d = overlap;
    const int i0 = bi * sub[0], i1 = i0 + sub[0], j0 = bj * sub[1], j1 = j0 + sub[1];
    const int k0 = bk * sub[2], k1 = k0 + sub[2];
    for (int k = k0 - d; k < k1 + d; ++k)
        for (int j = j0 - d; j < j1 + d; ++j)
            for (int i = i0 - d; i < i1 + d; ++i) {
                const int64_t c = box_cell(g, p, i, j, k);
                if (c < 0) continue;
                const bool owned = i >= i0 && i < i1 && j >= j0 && j < j1 && k >= k0 && k < k1;
                g2l[c] = int32_t(L.gcell.size());
                if (owned) L.own.push_back(int32_t(L.gcell.size()));
                L.gcell.push_back(int32_t(c));
            }
    const int64_t nloc = int64_t(L.gcell.size()), nrow = 4 * nloc;
    L.rp.assign(nrow + 1, 0);
    TermVec terms;
    std::vector<std::pair<int32_t, double>> loc;
    for (int64_t l = 0; l < nloc; ++l) {
        const int64_t gc = L.gcell[l];
        const int ii = int(gc % g.n), jj = int((gc / g.n) % g.n), kk = int((gc / (int64_t(g.n) * g.n)) % g.nr);
        const int pp = int(gc / (int64_t(g.n) * g.n * g.nr));
        for (int c = 0; c < 4; ++c) {
            terms.clear();
            Expander ex(g, op, terms);
            ex.row(pp, ii, jj, kk, c);
            loc.clear();
            for (auto &t : terms) {
                const int32_t lc = g2l[t.first / 4];
                if (lc >= 0) loc.emplace_back(4 * lc + int32_t(t.first % 4), t.second);
            }
            std::sort(loc.begin(), loc.end(), [](auto &a, auto &b) { return a.first < b.first; });
            size_t m = 0;
            for (size_t a = 0; a < loc.size(); ++a) {
                if (m > 0 && loc[m - 1].first == loc[a].first) loc[m - 1].second += loc[a].second;
                else loc[m++] = loc[a];
            }
            for (size_t a = 0; a < m; ++a) { L.ci.push_back(loc[a].first); L.v.push_back(loc[a].second); }
            L.rp[4 * l + c + 1] = int64_t(L.ci.size());
        }
    }
    for (int32_t c : L.gcell) g2l[c] = -1;
    L.owned_row.assign(L.gcell.size(), 0);
    for (int32_t l : L.own) L.owned_row[l] = 1;

    // ILU(0): for each row i, for each k < i in the row: l_ik = a_ik / u_kk,
    // then a_ij -= l_ik u_kj for the j > k present in row i.
    L.diag.assign(nrow, -1);
    std::vector<int64_t> pos(nrow, -1);
    for (int64_t r = 0; r < nrow; ++r) {
        for (int64_t q = L.rp[r]; q < L.rp[r + 1]; ++q) {
            pos[L.ci[q]] = q;
            if (L.ci[q] == r) L.diag[r] = q;
        }
        if (L.diag[r] < 0) { L.status = CSDYN_EZEROPIVOT; return; }
        for (int64_t q = L.rp[r]; q < L.diag[r]; ++q) {
            const int64_t kr = L.ci[q];
            const double lik = L.v[q] / L.v[L.diag[kr]];
            L.v[q] = lik;
            for (int64_t u = L.diag[kr] + 1; u < L.rp[kr + 1]; ++u) {
                const int64_t at = pos[L.ci[u]];
                if (at >= 0) L.v[at] -= lik * L.v[u];
            }
        }
        for (int64_t q = L.rp[r]; q < L.rp[r + 1]; ++q) pos[L.ci[q]] = -1;
        if (!(std::fabs(L.v[L.diag[r]]) >= 1e-300)) { L.status = CSDYN_EZEROPIVOT; return; }
    }
    // level schedules (longest path in the dependency DAG of each sweep)
    L.levL.assign(nrow, 0);
    L.levU.assign(nrow, 0);
    for (int64_t r = 0; r < nrow; ++r) {
        int lv = 0;
        for (int64_t q = L.rp[r]; q < L.diag[r]; ++q) lv = std::max(lv, L.levL[L.ci[q]] + 1);
        L.levL[r] = lv;
        L.nlevL = std::max(L.nlevL, lv + 1);
    }
    for (int64_t r = nrow - 1; r >= 0; --r) {
        int lv = 0;
        for (int64_t q = L.diag[r] + 1; q < L.rp[r + 1]; ++q) lv = std::max(lv, L.levU[L.ci[q]] + 1);
        L.levU[r] = lv;
        L.nlevU = std::max(L.nlevU, lv + 1);
    }
}

// Row schedule of one sweep of one subdomain: rows by level, within a level
// by decreasing width, cut into slices of 64 lanes.  A row with more than
// kLaneEntries entries is split over s = ceil(width / kLaneEntries) adjacent
// lanes in parts of ceil(width / s) entries (lane j of the row takes entries
// [j * part, (j + 1) * part)); a slice holds floor(64 / s) rows of one split.
constexpr int kLaneEntries = 8;

struct Schedule {
    std::vector<int32_t> lev_first;   // [nlev + 1] first slice (relative) of each level
    std::vector<int32_t> slice_rows;  // [nslice * 64] row held by each lane or -1
    std::vector<int32_t> slice_s;     // [nslice] lanes per row
    std::vector<int32_t> slice_nrow;  // [nslice] rows in the slice
    std::vector<int32_t> slice_slot;  // [nslice] ring slot of the slice's first row
    std::vector<int32_t> pos;         // [nrow] slice*64 + the row's index in its slice (relative)
    std::vector<int32_t> slot;        // [nrow] ring slot
};

// Ring addressing (depth > 0): slot = (level mod depth) * width + position in
// the level.  Box-vector addressing (depth == 0): the L sweep's slot is the
// row's position in the L sweep's order (levels one after another), and the U
// sweep addresses rows by the L sweep's slots (lslot).
void make_schedule(const LocalSd &L, bool upper, int depth, int width, const std::vector<int32_t> *lslot,
                   Schedule &S) {
    const int64_t nrow = int64_t(L.rp.size()) - 1;
    const int nlev = upper ? L.nlevU : L.nlevL;
    const std::vector<int32_t> &lev = upper ? L.levU : L.levL;
    auto cnt = [&](int64_t r) -> int64_t { return upper ? L.rp[r + 1] - L.diag[r] - 1 : L.diag[r] - L.rp[r]; };
    std::vector<std::vector<int32_t>> rows(nlev);
    for (int64_t r = 0; r < nrow; ++r) rows[lev[r]].push_back(int32_t(r));
    S.lev_first.assign(1, 0);
    S.slice_rows.clear();
    S.slice_s.clear();
    S.slice_nrow.clear();
    S.slice_slot.clear();
    S.pos.assign(nrow, -1);
    S.slot.assign(nrow, -1);
    int64_t cum = 0;  // rows of the previous levels
    auto slot_of = [&](int lv, int64_t a, int32_t r) -> int32_t {
        if (depth > 0) return int32_t((lv % depth) * width + a);
        return lslot ? (*lslot)[r] : int32_t(cum + a);
    };
    for (int lv = 0; lv < nlev; ++lv) {
        auto &R = rows[lv];
        std::stable_sort(R.begin(), R.end(), [&](int32_t a, int32_t b) { return cnt(a) > cnt(b); });
        int nsl = 0;
        for (size_t a = 0; a < R.size();) {
            const int sp = int(std::min<int64_t>(64, std::max<int64_t>(1, (cnt(R[a]) + kLaneEntries - 1) / kLaneEntries)));
            const int nr = int(std::min<size_t>(size_t(64 / sp), R.size() - a));
            const int sl = int(S.slice_s.size());
            S.slice_s.push_back(sp);
            S.slice_nrow.push_back(nr);
            S.slice_slot.push_back(lslot ? -1 : slot_of(lv, int64_t(a), R[a]));
            for (int l = 0; l < 64; ++l) {
                const int rr = l / sp;
                S.slice_rows.push_back(rr < nr ? R[a + rr] : -1);
            }
            for (int rr = 0; rr < nr; ++rr) {
                S.pos[R[a + rr]] = sl * 64 + rr;
                S.slot[R[a + rr]] = slot_of(lv, int64_t(a) + rr, R[a + rr]);
            }
            a += nr;
            ++nsl;
        }
        S.lev_first.push_back(S.lev_first.back() + nsl);
        cum += int64_t(R.size());
    }
}

// Append one subdomain's sweep to the pack.  Ring addressing: U_sched is the
// U schedule (for the L sweep's lane_next), base_u its first global U slice.
// Box-vector addressing (box_vector): lane_next is the row's position in the
// box vector (its L-sweep slot) in both sweeps.
int32_t pack_sweep(const LocalSd &L, bool upper, const Schedule &S, const Schedule *U_sched, int64_t base_u,
                   bool box_vector, SweepPack &P, int32_t &lev0, int32_t &lev1) {
    auto first = [&](int64_t r) { return upper ? L.diag[r] + 1 : L.rp[r]; };
    auto cnt = [&](int64_t r) -> int64_t { return upper ? L.rp[r + 1] - L.diag[r] - 1 : L.diag[r] - L.rp[r]; };
    const int64_t base = int64_t(P.sl_info.size());
    lev0 = int32_t(P.lev_slice.size());
    for (size_t lv = 0; lv + 1 < S.lev_first.size(); ++lv) P.lev_slice.push_back(int32_t(base + S.lev_first[lv]));
    lev1 = int32_t(P.lev_slice.size());
    const int nsl = S.lev_first.back();
    const int64_t pair0 = int64_t(P.val.size()) / 2;
    for (int sl = 0; sl < nsl; ++sl) {
        const int sp = S.slice_s[sl];
        const int32_t r0 = S.slice_rows[sl * 64];
        const int w = int((cnt(r0) + sp - 1) / sp);  // entries per lane
        if (w > kLaneEntries) {
            set_error("ras: a factor row has more than %d entries", 64 * kLaneEntries);
            return CSDYN_EINVAL;
        }
        const int64_t off = int64_t(P.val.size()) / 2, aoff = int64_t(P.addr.size()) / 8;
        P.sl_info.push_back(S.slice_nrow[sl] << 10 | (sp - 1) << 4 | w);
        P.sl_off.push_back(off);
        P.sl_slot.push_back(S.slice_slot[sl]);
        // full pairs [w / 2][64 lanes]; an odd width's last entry as one value per lane [64] after them
        const int np = w / 2;
        P.val.resize(P.val.size() + size_t(np) * 128 + (w % 2) * 64, 0.0);
        P.addr.resize(P.addr.size() + 512, 0);
        auto vat = [&](int64_t q, int a) {
            return q < 2 * np ? 2 * (off + (q / 2) * 64 + a) + q % 2 : 2 * (off + int64_t(np) * 64) + a;
        };
        auto aat = [&](int64_t q, int a) { return 8 * (aoff + a) + q; };
        for (int a = 0; a < 64; ++a) {
            const int32_t r = S.slice_rows[sl * 64 + a];
            int32_t io = -1, nxt = -1;
            double dg = 0.0;
            if (r >= 0) {
                const int j = a % sp;  // part of the row on this lane
                if (upper) {
                    dg = L.v[L.diag[r]];
                    if (j == 0 && L.owned_row[r / 4]) io = int32_t(4 * int64_t(L.gcell[r / 4]) + r % 4);
                    if (j == 0 && box_vector) nxt = S.slot[r];
                } else if (j == 0) {
                    io = int32_t(4 * int64_t(L.gcell[r / 4]) + r % 4);
                    nxt = box_vector ? S.slot[r] : int32_t(base_u * 64 + U_sched->pos[r]);
                }
                const int64_t q0 = first(r), n = cnt(r);
                for (int e = 0; e < kLaneEntries; ++e) {
                    const int64_t t = int64_t(j) * w + e;
                    if (e < w && t < n) {
                        P.val[vat(e, a)] = L.v[q0 + t];
                        P.addr[aat(e, a)] = uint16_t(S.slot[L.ci[q0 + t]]);
                    } else {
                        P.addr[aat(e, a)] = uint16_t(S.slot[r]);  // zero value
                    }
                }
            }
            P.lane_io.push_back(io);
            if (!upper || box_vector) P.lane_next.push_back(nxt);
            if (upper) P.lane_diag.push_back(dg);
        }
        if (upper || !box_vector) {  // per row of the slice (slice*64 + row), not per lane: the U sweep's u_ii
                                     // and slot (box vector) or y index (ring), the ring L sweep's x index and U row
            const size_t b = P.lane_io.size() - 64;
            for (int rr = 0; rr < 64; ++rr) {
                const int32_t r = rr < S.slice_nrow[sl] ? S.slice_rows[sl * 64 + rr * sp] : -1;
                const int32_t xi = r >= 0 ? int32_t(4 * int64_t(L.gcell[r / 4]) + r % 4) : -1;
                if (upper) {
                    P.lane_diag[b + size_t(rr)] = r >= 0 ? L.v[L.diag[r]] : 0.0;
                    if (box_vector) P.lane_next[b + size_t(rr)] = r >= 0 ? S.slot[r] : -1;
                    else P.lane_io[b + size_t(rr)] = r >= 0 && L.owned_row[r / 4] ? xi : -1;
                } else {
                    P.lane_io[b + size_t(rr)] = xi;
                    P.lane_next[b + size_t(rr)] = r >= 0 ? int32_t(base_u * 64 + U_sched->pos[r]) : -1;
                }
            }
        }
    }
    if (int64_t(P.val.size()) / 2 - pair0 > INT32_MAX) {  // the sweep kernel keeps 32-bit offsets per subdomain
        set_error("ras: subdomain too large (more than 2^31 value pairs in one sweep)");
        return CSDYN_EINVAL;
    }
    return CSDYN_OK;
}

// Longest distance in levels between a row and its dependencies, and the
// largest number of rows in one level, over both sweeps.
void sweep_stats(const LocalSd &L, int &span, int &rows) {
    const int64_t nrow = int64_t(L.rp.size()) - 1;
    span = 0;
    rows = 0;
    for (int upper = 0; upper < 2; ++upper) {
        const std::vector<int32_t> &lev = upper ? L.levU : L.levL;
        std::vector<int32_t> count(upper ? L.nlevU : L.nlevL, 0);
        for (int64_t r = 0; r < nrow; ++r) {
            ++count[lev[r]];
            const int64_t a = upper ? L.diag[r] + 1 : L.rp[r], b = upper ? L.rp[r + 1] : L.diag[r];
            for (int64_t q = a; q < b; ++q) span = std::max(span, lev[r] - lev[L.ci[q]]);
        }
        for (int32_t c : count) rows = std::max(rows, int(c));
    }
}

// Fold point and the level after which the late inputs are written, for one
// subdomain whose box vector gets at most `cap` slots (HostRas::folded gives
// the conditions).  S: the L schedule (box-vector positions).  Returns false
// when no slice boundary within cap satisfies them.
bool fold_plan(const LocalSd &L, const Schedule &S, int cap, int max_late, int32_t &fold, int32_t &fold_lev,
               int32_t &fold_levU) {
    const int nrow = int(L.rp.size()) - 1;
    fold = nrow;
    fold_lev = fold_levU = -1;
    if (nrow <= cap) return true;
    int f = 0;  // the largest slice start within cap
    for (int32_t p0 : S.slice_slot)
        if (p0 <= cap) f = std::max(f, int(p0));
    const int early = nrow - f;
    if (f <= 0 || early > f || early > max_late) return false;
    // last level at which each row is read or written, per sweep
    std::vector<int32_t> lastL(L.levL), lastU(L.levU);
    for (int d = 0; d < nrow; ++d) {
        for (int64_t q = L.rp[d]; q < L.diag[d]; ++q) lastL[L.ci[q]] = std::max(lastL[L.ci[q]], L.levL[d]);
        for (int64_t q = L.diag[d] + 1; q < L.rp[d + 1]; ++q) lastU[L.ci[q]] = std::max(lastU[L.ci[q]], L.levU[d]);
    }
    int aL = -1, bL = INT32_MAX, aU = -1, bU = INT32_MAX;
    for (int r = 0; r < nrow; ++r) {
        const int p = S.slot[r];
        if (p < early) {
            aL = std::max(aL, int(lastL[r]));
            bU = std::min(bU, int(L.levU[r]));
        }
        if (p >= f) {
            bL = std::min(bL, int(L.levL[r]));
            aU = std::max(aU, int(lastU[r]));
        }
    }
    if (bL < aL + 2 || bU < aU + 2) return false;
    fold = f;
    fold_lev = aL;
    fold_levU = aU;
    return true;
}

}  // namespace

// ------------------------------------------------------------------ padded value layout
constexpr int64_t kTailPairs = 64 * 64 / 2;  // the pairs of the tail padding after the last slice

std::vector<int64_t> padded_offsets(const SweepPack &P) {
    std::vector<int64_t> off(P.sl_info.size() + 1);
    int64_t cur = 0;
    for (size_t sl = 0; sl < P.sl_info.size(); ++sl) {
        off[sl] = cur;
        cur += int64_t((P.sl_info[sl] & 15) + 1) / 2 * 64;
    }
    off.back() = cur;
    return off;
}

int64_t padded_pairs(const SweepPack &P) { return padded_offsets(P).back() + kTailPairs; }

template <class T>
void padded_values(const SweepPack &P, const std::vector<int64_t> &new_off, T *out) {
    const int64_t nsl = int64_t(P.sl_info.size());
    std::fill(out + 2 * new_off[size_t(nsl)], out + 2 * (new_off[size_t(nsl)] + kTailPairs), T(0));
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t sl = 0; sl < nsl; ++sl) {
        const int w = P.sl_info[size_t(sl)] & 15, np = w / 2;
        const double *src = P.val.data() + 2 * P.sl_off[size_t(sl)];
        T *dst = out + 2 * new_off[size_t(sl)];
        for (int64_t a = 0; a < int64_t(np) * 128; ++a) dst[a] = T(src[a]);
        if (w % 2)
            for (int a = 0; a < 64; ++a) {
                dst[int64_t(np) * 128 + 2 * a] = T(src[int64_t(np) * 128 + a]);
                dst[int64_t(np) * 128 + 2 * a + 1] = T(0);
            }
    }
}
template void padded_values<float>(const SweepPack &, const std::vector<int64_t> &, float *);
template void padded_values<double>(const SweepPack &, const std::vector<int64_t> &, double *);

void padded_meta(const HostRas &H, const std::vector<int32_t> &Lsrc, const std::vector<int64_t> &Loff,
                 const std::vector<int64_t> &Uoff, std::vector<SdInfo> &sd, std::vector<int32_t> &Lmeta,
                 std::vector<int32_t> &Umeta) {
    sd = H.sd;
    Lmeta = Lsrc;
    Umeta = H.U.meta;
    const int offw = int(((size_t(H.max_levels) + 1) * 4 + 15) / 16 * 16 / 4);
    for (int s = 0; s < H.nsd; ++s) {
        SdInfo &I = sd[size_t(s)];
        for (int pass = 0; pass < 2; ++pass) {
            const std::vector<int64_t> &no = pass ? Uoff : Loff;
            const int sl0 = pass ? I.slU0 : I.slL0, nsl = pass ? I.nslU : I.nslL;
            const int64_t off0 = nsl > 0 ? no[size_t(sl0)] : 0;
            (pass ? I.offU0 : I.offL0) = off0;
            int32_t *m = (pass ? Umeta : Lmeta).data() + size_t(s) * H.meta_words;
            for (int q = 0; q < nsl; ++q) m[offw + q] = int32_t(no[size_t(sl0 + q)] - off0);
        }
    }
}

int32_t host_subdomain(const HostGeom &g, const csdyn_op &op, const int sub[3], int overlap, int s,
                       std::vector<int32_t> &gcell, std::vector<int32_t> &own, std::vector<int64_t> &rp,
                       std::vector<int32_t> &ci, std::vector<double> &v) {
    if (sub[0] < 1 || sub[1] < 1 || sub[2] < 1 || g.n % sub[0] || g.n % sub[1] || g.nr % sub[2] || overlap < 0 ||
        overlap > 1) {
        set_error("ras: bad subdomain size or overlap");
        return CSDYN_EINVAL;
    }
    const int nb[3] = {g.n / sub[0], g.n / sub[1], g.nr / sub[2]};
    if (s < 0 || s >= 6 * nb[0] * nb[1] * nb[2]) { set_error("ras: subdomain index out of range"); return CSDYN_EINVAL; }
    std::vector<int32_t> g2l(6 * int64_t(g.n) * g.n * g.nr, -1);
    LocalSd L;
    build_one(g, op, sub, nb, overlap, s, g2l, L);
    if (L.status != CSDYN_OK) { set_error("ras: zero pivot in subdomain %d", s); return L.status; }
    gcell.swap(L.gcell); own.swap(L.own); rp.swap(L.rp); ci.swap(L.ci); v.swap(L.v);
    return CSDYN_OK;
}

void stencil_row(const HostGeom &g, const csdyn_op &op, int p, int i, int j, int k, int c, TermVec &out) {
    Expander ex(g, op, out);
    ex.row(p, i, j, k, c);
}

int32_t build_host_ras(const HostGeom &g, const csdyn_op &op, const int sub[3], int overlap, int storage,
                       HostRas &H) {
    if (sub[0] < 1 || sub[1] < 1 || sub[2] < 1 || g.n % sub[0] || g.n % sub[1] || g.nr % sub[2]) {
        set_error("ras: grid %dx%dx%d is not divisible by subdomain %dx%dx%d", g.n, g.n, g.nr, sub[0], sub[1], sub[2]);
        return CSDYN_EINVAL;
    }
    if (overlap < 0 || overlap > 1) { set_error("ras: overlap must be 0 or 1"); return CSDYN_EINVAL; }
    H = HostRas();
    H.nb[0] = g.n / sub[0]; H.nb[1] = g.n / sub[1]; H.nb[2] = g.nr / sub[2];
    H.nsd = 6 * H.nb[0] * H.nb[1] * H.nb[2];
    std::vector<LocalSd> loc(H.nsd);
    const int64_t ncell = 6 * int64_t(g.n) * g.n * g.nr;
    int32_t status = CSDYN_OK;
#pragma omp parallel
    {
        std::vector<int32_t> g2l(ncell, -1);
#pragma omp for schedule(dynamic, 1)
        for (int s = 0; s < H.nsd; ++s) build_one(g, op, sub, H.nb, overlap, s, g2l, loc[s]);
    }
    for (int s = 0; s < H.nsd; ++s)
        if (loc[s].status != CSDYN_OK) {
            status = loc[s].status;
            set_error("ras: zero pivot in the ILU(0) factorization of subdomain %d", s);
            return status;
        }
    // ring geometry shared by all subdomains
    int span = 0, rows = 0;
    for (int s = 0; s < H.nsd; ++s) {
        int sp, rw;
        sweep_stats(loc[s], sp, rw);
        span = std::max(span, sp);
        rows = std::max(rows, rw);
    }
    H.ring_depth = span + 1;
    H.ring_width = ((rows + 63) / 64) * 64;
    for (int s = 0; s < H.nsd; ++s) H.box_rows = std::max(H.box_rows, int(loc[s].rp.size()) - 1);
    if (storage < 0 || storage > 3) { set_error("ras: storage must be 0, 1, 2 or 3"); return CSDYN_EINVAL; }
    const int64_t vec_bytes = int64_t(H.box_rows) * int64_t(sizeof(double));
    const int max_late = kFoldRegs * sweep_threads(H.ring_width);
    // A subdomain vector above the automatic bound can still live in LDS folded
    // into one workgroup's share (kLdsFoldBytes) when its late rows fit the
    // registers that hold them; the schedules below decide.
    const bool try_big = (storage == 0 || storage == 2) && vec_bytes > kBoxVectorBytes &&
                         int64_t(H.box_rows) - kLdsFoldBytes / int64_t(sizeof(double)) <= max_late;
    H.box_vector = storage == 2 || (storage != 1 && vec_bytes <= kBoxVectorBytes) || try_big;
    if (H.box_vector && H.box_rows > 65535) {
        set_error("ras: subdomain of %d rows too large for 16-bit vector addresses", H.box_rows);
        return CSDYN_EINVAL;
    }
    // Folding: the metadata size needs every subdomain's slice counts first.
    int fold_cap = 0;
    if (H.box_vector && storage != 3) {
        int msl = 0, mlev = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(max : msl, mlev)
        for (int s = 0; s < H.nsd; ++s) {
            Schedule a, b;
            make_schedule(loc[s], false, 0, H.ring_width, nullptr, a);
            make_schedule(loc[s], true, 0, H.ring_width, &a.slot, b);
            msl = std::max(msl, std::max(a.lev_first.back(), b.lev_first.back()));
            mlev = std::max(mlev, std::max(loc[s].nlevL, loc[s].nlevU));
        }
        const int64_t meta = int64_t(meta_bytes_for(msl, mlev));
        const int64_t budget = vec_bytes <= kBoxVectorBytes ? kFoldBytes : kLdsFoldBytes;
        if (meta + vec_bytes > budget && meta < budget) fold_cap = int((budget - meta) / int64_t(sizeof(double)));
        if (try_big) {  // every subdomain must fold, else the ring (storage 0) or the setup error (storage 2)
            bool ok = fold_cap > 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(&& : ok)
            for (int s = 0; s < H.nsd; ++s) {
                if (!ok) continue;
                Schedule a;
                make_schedule(loc[s], false, 0, H.ring_width, nullptr, a);
                int32_t f, l, u;
                ok = ok && fold_plan(loc[s], a, fold_cap, max_late, f, l, u);
            }
            if (!ok) {
                fold_cap = 0;
                if (storage == 0) H.box_vector = false;
            }
        }
    }
    if (!H.box_vector && int64_t(H.ring_depth) * H.ring_width > 65536) {
        set_error("ras: subdomain too large for the level ring (%d levels x %d rows)", H.ring_depth, H.ring_width);
        return CSDYN_EINVAL;
    }
    H.folded = fold_cap > 0;
    // Schedules and packs: each subdomain's in parallel into a pack of its own
    // (slice, pair, lane and level indices from 0), then appended in subdomain
    // order with its offsets added, a chunk of subdomains at a time so that the
    // local packs never hold more than a chunk's data.
    struct Packed {
        SweepPack L, U;
        std::vector<int32_t> gio, fold_Upos, own;
        std::vector<uint16_t> fold_Laddr, fold_Uaddr;
        int32_t levL0 = 0, levL1 = 0, levU0 = 0, levU1 = 0;
        int32_t status = CSDYN_OK;
        std::string err;
        bool fold_ok = true;
        int max_slices = 0;
        int64_t nnz = 0;
    };
    const int depth = H.box_vector ? 0 : H.ring_depth;
    const bool want_fold = H.folded;
    constexpr int kChunk = 64;
    H.sd.resize(H.nsd);
    for (int c0 = 0; c0 < H.nsd; c0 += kChunk) {
        const int c1 = std::min(H.nsd, c0 + kChunk);
        std::vector<Packed> pk(size_t(c1 - c0));
#pragma omp parallel for schedule(dynamic, 1)
        for (int s = c0; s < c1; ++s) {
            LocalSd &L = loc[s];
            SdInfo &I = H.sd[s];
            Packed &Q = pk[size_t(s - c0)];
            const int64_t nrow = int64_t(L.rp.size()) - 1;
            I.nrows = int32_t(nrow);
            I.fold = int32_t(nrow);
            I.fold_lev = I.fold_levU = -1;
            I.nloc = int32_t(L.gcell.size());
            I.nown = int32_t(L.own.size());
            Q.nnz = int64_t(L.ci.size());
            Schedule SL, SU;
            make_schedule(L, false, depth, H.ring_width, nullptr, SL);
            make_schedule(L, true, depth, H.ring_width, H.box_vector ? &SL.slot : nullptr, SU);
            if (H.box_vector) {  // position SL.slot[r] of the box vector holds row r
                Q.gio.assign(size_t(nrow), -1);
                for (int64_t r = 0; r < nrow && Q.status == CSDYN_OK; ++r) {
                    const int64_t a = SL.slot[r];
                    if (a < 0 || a >= nrow || Q.gio[size_t(a)] >= 0) {
                        Q.status = CSDYN_EINVAL;
                        Q.err = "ras: box-vector positions of subdomain " + std::to_string(s) + " are not a permutation";
                    } else {
                        Q.gio[size_t(a)] = int32_t(4 * int64_t(L.gcell[r / 4]) + r % 4);
                    }
                }
            }
            if (want_fold) Q.fold_ok = fold_plan(L, SL, fold_cap, max_late, I.fold, I.fold_lev, I.fold_levU);
            if (H.box_vector) {  // owned rows {slot, y index}: the late ones (slots reused by the fold) first
                const int32_t f = want_fold && Q.fold_ok ? I.fold : int32_t(nrow);
                I.own_late = 0;
                for (int pass = 0; pass < 2; ++pass)
                    for (int64_t r = 0; r < nrow; ++r) {
                        if (!L.owned_row[size_t(r / 4)]) continue;
                        const int32_t p = SL.slot[size_t(r)];
                        if ((p >= f) != (pass == 0)) continue;
                        Q.own.push_back(p);
                        Q.own.push_back(int32_t(4 * int64_t(L.gcell[size_t(r / 4)]) + r % 4));
                        I.own_late += pass == 0;
                    }
            }
            int32_t e = Q.status;
            if (e == CSDYN_OK) e = pack_sweep(L, true, SU, nullptr, 0, H.box_vector, Q.U, Q.levU0, Q.levU1);
            if (e == CSDYN_OK) e = pack_sweep(L, false, SL, &SU, 0, H.box_vector, Q.L, Q.levL0, Q.levL1);
            if (e != CSDYN_OK && Q.status == CSDYN_OK) {
                Q.status = e;
                Q.err = csdyn_last_error();
            }
            if (e == CSDYN_OK && want_fold && Q.fold_ok) {  // the folded copies (parallel to the packs)
                const int32_t f = I.fold;
                auto slot = [&](int32_t p) { return p >= f ? p - f : p; };
                Q.fold_Uaddr.reserve(Q.U.addr.size());
                Q.fold_Laddr.reserve(Q.L.addr.size());
                for (uint16_t a : Q.U.addr) Q.fold_Uaddr.push_back(uint16_t(slot(a)));
                for (uint16_t a : Q.L.addr) Q.fold_Laddr.push_back(uint16_t(slot(a)));
                for (int32_t p : Q.U.lane_next) Q.fold_Upos.push_back(p < 0 ? -1 : slot(p));
            }
            Q.max_slices = std::max(SL.lev_first.back(), SU.lev_first.back());
            LocalSd().gcell.swap(L.gcell);
            std::vector<int64_t>().swap(L.rp);
            std::vector<int32_t>().swap(L.ci);
            std::vector<double>().swap(L.v);
        }
        // offsets of each subdomain of the chunk in the appended arrays (and the
        // bases its indices are shifted by), then the copies in parallel
        const int nc = c1 - c0;
        for (int q = 0; q < nc; ++q)
            if (pk[size_t(q)].status != CSDYN_OK) {
                set_error("%s", pk[size_t(q)].err.c_str());
                return pk[size_t(q)].status;
            }
        if (H.folded)
            for (int q = 0; q < nc; ++q) H.folded = H.folded && pk[size_t(q)].fold_ok;
        struct Off {
            size_t lev[2], sl[2], pair[2], lane[2], addr[2], gio, fpos, own;
        };
        std::vector<Off> off(size_t(nc) + 1);
        SweepPack *HP[2] = {&H.L, &H.U};
        for (int w = 0; w < 2; ++w) {
            off[0].lev[w] = HP[w]->lev_slice.size();
            off[0].sl[w] = HP[w]->sl_info.size();
            off[0].pair[w] = HP[w]->val.size() / 2;
            off[0].lane[w] = HP[w]->lane_io.size();
            off[0].addr[w] = HP[w]->addr.size();
        }
        off[0].gio = H.gio.size();
        off[0].fpos = H.fold_Upos.size();
        off[0].own = H.own.size();
        for (int q = 0; q < nc; ++q) {
            const Packed &Q = pk[size_t(q)];
            for (int w = 0; w < 2; ++w) {
                const SweepPack &P = w ? Q.U : Q.L;
                off[size_t(q) + 1].lev[w] = off[size_t(q)].lev[w] + P.lev_slice.size();
                off[size_t(q) + 1].sl[w] = off[size_t(q)].sl[w] + P.sl_info.size();
                off[size_t(q) + 1].pair[w] = off[size_t(q)].pair[w] + P.val.size() / 2;
                off[size_t(q) + 1].lane[w] = off[size_t(q)].lane[w] + P.lane_io.size();
                off[size_t(q) + 1].addr[w] = off[size_t(q)].addr[w] + P.addr.size();
            }
            off[size_t(q) + 1].gio = off[size_t(q)].gio + Q.gio.size();
            off[size_t(q) + 1].own = off[size_t(q)].own + Q.own.size();
            off[size_t(q) + 1].fpos = off[size_t(q)].fpos + (H.folded ? Q.fold_Upos.size() : 0);
        }
        // the first chunk sets the capacity of the whole build (no reallocation
        // copies later unless later subdomains are larger)
        auto grow = [&](auto &v, size_t n) {
            if (c0 == 0) v.reserve(size_t(double(n) * double(H.nsd) / double(nc) * 1.05) + 64 * 64);
            v.resize(n);
        };
        for (int w = 0; w < 2; ++w) {
            SweepPack &P = *HP[w];
            grow(P.lev_slice, off[size_t(nc)].lev[w]);
            grow(P.sl_info, off[size_t(nc)].sl[w]);
            grow(P.sl_off, off[size_t(nc)].sl[w]);
            grow(P.sl_slot, off[size_t(nc)].sl[w]);
            grow(P.lane_io, off[size_t(nc)].lane[w]);
            if (w == 0 || H.box_vector) grow(P.lane_next, off[size_t(nc)].lane[w]);
            if (w == 1) grow(P.lane_diag, off[size_t(nc)].lane[w]);
            grow(P.val, 2 * off[size_t(nc)].pair[w]);
            grow(P.addr, off[size_t(nc)].addr[w]);
        }
        grow(H.gio, off[size_t(nc)].gio);
        grow(H.own, off[size_t(nc)].own);
        if (H.folded) {
            grow(H.fold_Laddr, off[size_t(nc)].addr[0]);
            grow(H.fold_Uaddr, off[size_t(nc)].addr[1]);
            grow(H.fold_Upos, off[size_t(nc)].fpos);
        }
#pragma omp parallel for schedule(dynamic, 1)
        for (int q = 0; q < nc; ++q) {
            Packed &Q = pk[size_t(q)];
            const Off &o = off[size_t(q)];
            SdInfo &I = H.sd[size_t(c0 + q)];
            for (int w = 0; w < 2; ++w) {
                SweepPack &P = *HP[w], &S = w ? Q.U : Q.L;
                for (size_t a = 0; a < S.lev_slice.size(); ++a) P.lev_slice[o.lev[w] + a] = int32_t(S.lev_slice[a] + o.sl[w]);
                std::copy(S.sl_info.begin(), S.sl_info.end(), P.sl_info.begin() + ptrdiff_t(o.sl[w]));
                for (size_t a = 0; a < S.sl_off.size(); ++a) P.sl_off[o.sl[w] + a] = S.sl_off[a] + int64_t(o.pair[w]);
                std::copy(S.sl_slot.begin(), S.sl_slot.end(), P.sl_slot.begin() + ptrdiff_t(o.sl[w]));
                std::copy(S.lane_io.begin(), S.lane_io.end(), P.lane_io.begin() + ptrdiff_t(o.lane[w]));
                // the ring's L lanes point at U lanes: shift them by this subdomain's first U lane
                const bool ring_l = w == 0 && !H.box_vector;
                const int64_t ub = int64_t(o.sl[1]) * 64;
                for (size_t a = 0; a < S.lane_next.size(); ++a)
                    P.lane_next[o.lane[w] + a] = ring_l && S.lane_next[a] >= 0 ? int32_t(S.lane_next[a] + ub) : S.lane_next[a];
                std::copy(S.lane_diag.begin(), S.lane_diag.end(), P.lane_diag.begin() + ptrdiff_t(o.lane[w]));
                std::copy(S.val.begin(), S.val.end(), P.val.begin() + ptrdiff_t(2 * o.pair[w]));
                std::copy(S.addr.begin(), S.addr.end(), P.addr.begin() + ptrdiff_t(o.addr[w]));
            }
            I.levL0 = Q.levL0 + int32_t(o.lev[0]);
            I.levL1 = Q.levL1 + int32_t(o.lev[0]);
            I.levU0 = Q.levU0 + int32_t(o.lev[1]);
            I.levU1 = Q.levU1 + int32_t(o.lev[1]);
            I.g0 = int64_t(o.gio);
            std::copy(Q.gio.begin(), Q.gio.end(), H.gio.begin() + ptrdiff_t(o.gio));
            I.own0 = int64_t(o.own / 2);
            std::copy(Q.own.begin(), Q.own.end(), H.own.begin() + ptrdiff_t(o.own));
            if (H.folded) {
                std::copy(Q.fold_Laddr.begin(), Q.fold_Laddr.end(), H.fold_Laddr.begin() + ptrdiff_t(o.addr[0]));
                std::copy(Q.fold_Uaddr.begin(), Q.fold_Uaddr.end(), H.fold_Uaddr.begin() + ptrdiff_t(o.addr[1]));
                std::copy(Q.fold_Upos.begin(), Q.fold_Upos.end(), H.fold_Upos.begin() + ptrdiff_t(o.fpos));
            }
        }
        for (int q = 0; q < nc; ++q) {
            Packed &Q = pk[size_t(q)];
            const LocalSd &L = loc[size_t(c0 + q)];
            const SdInfo &I = H.sd[size_t(c0 + q)];
            H.box_cells += I.nloc;
            H.owned_cells += I.nown;
            H.nnz += Q.nnz;
            if (H.folded) {
                H.fold_rows = std::max(H.fold_rows, int(I.fold));
                H.fold_early = std::max(H.fold_early, int(I.nrows - I.fold));
            }
            H.max_slices = std::max(H.max_slices, Q.max_slices);
            H.max_levels = std::max(H.max_levels, std::max(L.nlevL, L.nlevU));
            H.max_total_levels = std::max(H.max_total_levels, L.nlevL + L.nlevU);
            Q = Packed();
        }
    }
    if (H.max_levels >= 1 << 14) {
        set_error("ras: %d levels in one triangular sweep (at most 16383)", H.max_levels);
        return CSDYN_EINVAL;
    }
    H.L.lev_slice.push_back(int32_t(H.L.sl_info.size()));
    H.U.lev_slice.push_back(int32_t(H.U.sl_info.size()));
    // per-subdomain metadata images, laid out as the sweep kernel's LDS copy
    H.meta_words = int(meta_bytes_for(H.max_slices, H.max_levels) / 4);
    const int offw = int(((size_t(H.max_levels) + 1) * 4 + 15) / 16 * 16 / 4), msl = H.max_slices;
    for (int pass = 0; pass < 2; ++pass) {
        SweepPack &P = pass ? H.U : H.L;
        P.meta.assign(size_t(H.nsd) * H.meta_words, 0);
        for (int s = 0; s < H.nsd; ++s) {
            SdInfo &I = H.sd[s];
            const int lev0 = pass ? I.levU0 : I.levL0, lev1 = pass ? I.levU1 : I.levL1;
            const int sl0 = P.lev_slice[lev0], nsl = P.lev_slice[lev1] - sl0;
            const int64_t off0 = nsl > 0 ? P.sl_off[sl0] : 0;
            (pass ? I.slU0 : I.slL0) = sl0;
            (pass ? I.nslU : I.nslL) = nsl;
            (pass ? I.offU0 : I.offL0) = off0;
            int32_t *m = P.meta.data() + size_t(s) * H.meta_words;
            for (int a = 0; a <= lev1 - lev0; ++a) m[a] = P.lev_slice[lev0 + a] - sl0;
            for (int a = 0; a < lev1 - lev0; ++a)
                for (int q = m[a]; q < m[a + 1]; ++q) m[offw + msl + q] = a << 17 | P.sl_info[sl0 + q];
            for (int q = 0; q < nsl; ++q) {
                m[offw + q] = int32_t(P.sl_off[sl0 + q] - off0);
                m[offw + 2 * msl + q] = P.sl_slot[sl0 + q];
            }
        }
    }
    if (H.folded) {  // the L sweep's slice slots, folded
        H.fold_Lmeta = H.L.meta;
        const int msl = H.max_slices;
        for (int s = 0; s < H.nsd; ++s) {
            const SdInfo &I = H.sd[s];
            int32_t *m = H.fold_Lmeta.data() + size_t(s) * H.meta_words;
            for (int q = 0; q < I.nslL; ++q) {
                int32_t &v = m[offw + 2 * msl + q];
                if (v >= I.fold) v -= I.fold;
            }
        }
    }
    // Boxes of the same shape at the same place relative to the panel edges and
    // the radial ends have the same sweep structure: each distinct address block
    // is stored once and the subdomains point at it.
    std::vector<int32_t> cls(H.nsd, 0);
    for (int pass = 0; pass < 2; ++pass) {
        SweepPack &P = pass ? H.U : H.L;
        constexpr size_t kSl = 8 * 64;  // addresses per slice
        std::vector<uint16_t> shared;
        std::map<std::pair<uint64_t, int>, std::vector<int32_t>> stored;  // (hash, slices) -> first slices
        std::vector<uint64_t> hs(H.nsd);
#pragma omp parallel for schedule(dynamic, 4)
        for (int s = 0; s < H.nsd; ++s) {
            const SdInfo &I = H.sd[s];
            const int sl0 = pass ? I.slU0 : I.slL0, nsl = pass ? I.nslU : I.nslL;
            const uint16_t *blk = P.addr.data() + size_t(sl0) * kSl;
            uint64_t h = 1469598103934665603ull;  // FNV-1a over the block
            for (size_t a = 0, len = size_t(nsl) * kSl; a < len; ++a) h = (h ^ blk[a]) * 1099511628211ull;
            hs[s] = h;
        }
        for (int s = 0; s < H.nsd; ++s) {
            SdInfo &I = H.sd[s];
            const int sl0 = pass ? I.slU0 : I.slL0, nsl = pass ? I.nslU : I.nslL;
            const uint16_t *blk = P.addr.data() + size_t(sl0) * kSl;
            const size_t len = size_t(nsl) * kSl;
            auto &cand = stored[{hs[s], nsl}];
            int32_t at = -1;
            for (int32_t c0 : cand)
                if (std::equal(blk, blk + len, shared.begin() + size_t(c0) * kSl)) { at = c0; break; }
            if (at < 0) {
                at = int32_t(shared.size() / kSl);
                shared.insert(shared.end(), blk, blk + len);
                cand.push_back(at);
            }
            (pass ? I.aslU0 : I.aslL0) = at;
        }
        if (H.folded) {  // the folded blocks, shared the same way (equal structures fold alike)
            std::vector<uint16_t> &F = pass ? H.fold_Uaddr : H.fold_Laddr;
            std::vector<uint16_t> fshared;
            for (int s = 0; s < H.nsd && H.folded; ++s) {
                const SdInfo &I = H.sd[s];
                const int sl0 = pass ? I.slU0 : I.slL0, nsl = pass ? I.nslU : I.nslL;
                const size_t at = size_t(pass ? I.aslU0 : I.aslL0) * kSl, len = size_t(nsl) * kSl;
                const uint16_t *blk = F.data() + size_t(sl0) * kSl;
                if (at == fshared.size()) fshared.insert(fshared.end(), blk, blk + len);
                else if (at + len > fshared.size() || !std::equal(blk, blk + len, fshared.begin() + at))
                    H.folded = false;
            }
            F.swap(fshared);
        }
        P.addr.swap(shared);
    }
    {
        std::map<std::pair<int32_t, int32_t>, int32_t> ids;
        for (int s = 0; s < H.nsd; ++s) {
            auto it = ids.emplace(std::make_pair(H.sd[s].aslL0, H.sd[s].aslU0), int32_t(ids.size())).first;
            cls[s] = it->second;
        }
        H.addr_classes = int(ids.size());
        // subdomains by structure, dealt to the L2 domains in runs
        std::vector<int32_t> bycls(H.nsd);
        std::iota(bycls.begin(), bycls.end(), 0);
        std::stable_sort(bycls.begin(), bycls.end(), [&](int32_t a, int32_t b) { return cls[a] < cls[b]; });
        H.perm.assign(H.nsd, -1);
        size_t q = 0;
        for (int x = 0; x < kXcds; ++x)
            for (int b = x; b < H.nsd; b += kXcds) H.perm[b] = bycls[q++];
    }
    // tail padding: the sweep kernel may read a fixed number of entries past a
    // slice's width; keep those reads inside the arrays
    for (SweepPack *P : {&H.L, &H.U}) {
        P->val.resize(P->val.size() + 64 * 64, 0.0);
        P->addr.resize(P->addr.size() + 64 * 64, 0);
    }
    if (H.folded) {
        H.fold_Laddr.resize(H.fold_Laddr.size() + 64 * 64, 0);
        H.fold_Uaddr.resize(H.fold_Uaddr.size() + 64 * 64, 0);
    } else {  // not needed, or some subdomain's levels do not allow it
        for (SdInfo &I : H.sd) {
            I.fold = I.nrows;
            I.fold_lev = I.fold_levU = -1;
        }
        H.fold_rows = H.fold_early = 0;
        std::vector<uint16_t>().swap(H.fold_Laddr);
        std::vector<uint16_t>().swap(H.fold_Uaddr);
        std::vector<int32_t>().swap(H.fold_Lmeta);
        std::vector<int32_t>().swap(H.fold_Upos);
    }
    return CSDYN_OK;
}

}  // namespace csd
