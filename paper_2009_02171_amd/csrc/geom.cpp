// Host-side geometry of the equiangular gnomonic cubed-sphere shell
// (Sec. 3.2): closed-form metric tables and the panel-edge tables.
//
// With X = tan xi, Y = tan eta, rho^2 = 1 + X^2 + Y^2 and the local frame
// (radial axis, then the xi and eta directions) the covariant basis of
// x = r (1, X, Y)/rho gives, in closed form,
//   sqrt(g)            = r^2 (1+X^2)(1+Y^2) / rho^3         (Sec. 3.2)
//   sqrt(g) g^11       = (1+Y^2)/rho,  sqrt(g) g^22 = (1+X^2)/rho,
//   sqrt(g) g^12       = X Y / rho                          (r-independent)
//   sqrt(g) g^1        = r (1+Y^2)(-X, 1, 0)/rho^2
//   sqrt(g) g^2        = r (1+X^2)(-Y, 0, 1)/rho^2
//   g^3 = g_3          = (1, X, Y)/rho,
//   r g^1 = rho (-X, 1, 0)/(1+X^2),  r g^2 = rho (-Y, 0, 1)/(1+Y^2).
// All six panels share the scalar tables; the vector tables are rotated by
// the panel's orientation.
#include <cmath>
#include <cstring>

#include "common.h"

namespace csd {

const int ROT[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},    // +x
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},   // +y
    {{-1, 0, 0}, {0, -1, 0}, {0, 0, 1}},  // -x
    {{0, 1, 0}, {-1, 0, 0}, {0, 0, 1}},   // -y
    {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},   // +z
    {{0, 0, 1}, {0, 1, 0}, {-1, 0, 0}},   // -z
};

static void to_global(int p, const double l[3], double g[3]) {
    for (int a = 0; a < 3; ++a) g[a] = ROT[p][a][0] * l[0] + ROT[p][a][1] * l[1] + ROT[p][a][2] * l[2];
}

static void to_local(int p, const double g[3], double l[3]) {
    for (int a = 0; a < 3; ++a) l[a] = ROT[p][0][a] * g[0] + ROT[p][1][a] * g[1] + ROT[p][2][a] * g[2];
}

// Extended (xi, eta) of panel edge e (0 W, 1 E, 2 S, 3 N) at tangential index
// t: the ghost-cell centre (depth 1) or the face centre (depth 1/2).
static void edge_coords(const HostGeom &g, int e, int t, double depth, double &xi, double &eta) {
    double lo = -depth, hi = g.n - 1 + depth;
    switch (e) {
        case 0: xi = g.ang(lo); eta = g.ang(t); break;
        case 1: xi = g.ang(hi); eta = g.ang(t); break;
        case 2: xi = g.ang(t); eta = g.ang(lo); break;
        default: xi = g.ang(t); eta = g.ang(hi); break;
    }
}

int32_t HostGeom::build(const csdyn_grid &g) {
    if (g.n < 4 || g.nr < 1 || !(g.ri > 0) || !(g.ro > g.ri)) {
        set_error("grid: need n >= 4, nr >= 1, 0 < ri < ro (got n=%d nr=%d ri=%g ro=%g)", g.n, g.nr, g.ri, g.ro);
        return CSDYN_EINVAL;
    }
    n = g.n; nr = g.nr; ri = g.ri; ro = g.ro;
    hs = 3.14159265358979323846 / (2.0 * n);
    hr = (ro - ri) / nr;
    ghost.assign(24 * size_t(n), GhostEntry{});
    face.assign(24 * size_t(n), FaceEntry{});
    const double qpi = 0.78539816339744830962;
    for (int p = 0; p < 6; ++p)
        for (int e = 0; e < 4; ++e)
            for (int t = 0; t < n; ++t) {
                // neighbour panel: the one whose centre axis is closest to the ghost point
                double xi, eta, loc[3], d[3];
                edge_coords(*this, e, t, 1.0, xi, eta);
                loc[0] = 1.0; loc[1] = std::tan(xi); loc[2] = std::tan(eta);
                to_global(p, loc, d);
                int q = -1;
                double best = -1.0;
                for (int c = 0; c < 6; ++c) {
                    double l2[3];
                    to_local(c, d, l2);
                    if (l2[0] > best) { best = l2[0]; q = c; }
                }
                double lq[3];
                to_local(q, d, lq);
                double aq = std::atan(lq[1] / lq[0]), bq = std::atan(lq[2] / lq[0]);
                GhostEntry &G = ghost[(p * 4 + e) * size_t(n) + t];
                G.q = q;
                double normal, tang;
                if (std::fabs(aq) > std::fabs(bq)) { G.fix_i = 1; normal = aq; tang = bq; }
                else { G.fix_i = 0; normal = bq; tang = aq; }
                double fidx = (normal + qpi) / hs - 0.5;
                G.idx = int(std::lround(fidx));
                if (std::fabs(fidx - G.idx) > 1e-8 || (G.idx != 0 && G.idx != n - 1)) {
                    set_error("grid: ghost of panel %d edge %d t %d is not on a first cell layer", p, e, t);
                    return CSDYN_EINVAL;
                }
                double s = (tang + qpi) / hs - 0.5;  // fractional index along the neighbour's line
                int m0 = int(std::floor(s)) - 1;
                m0 = m0 < 0 ? 0 : (m0 > n - 4 ? n - 4 : m0);
                G.m0 = m0;
                for (int m = 0; m < 4; ++m) {
                    double num = 1.0, den = 1.0;
                    for (int l = 0; l < 4; ++l) {
                        if (l == m) continue;
                        num *= s - double(m0 + l);
                        den *= double(m - l);
                    }
                    G.w[m] = num / den;
                }
                // the matching face on q
                edge_coords(*this, e, t, 0.5, xi, eta);
                loc[1] = std::tan(xi); loc[2] = std::tan(eta);
                to_global(p, loc, d);
                to_local(q, d, lq);
                aq = std::atan(lq[1] / lq[0]); bq = std::atan(lq[2] / lq[0]);
                FaceEntry &F = face[(p * 4 + e) * size_t(n) + t];
                F.q = q;
                double ft;
                if (std::fabs(std::fabs(aq) - qpi) < 1e-12) { F.e = aq < 0 ? 0 : 1; ft = (bq + qpi) / hs - 0.5; }
                else if (std::fabs(std::fabs(bq) - qpi) < 1e-12) { F.e = bq < 0 ? 2 : 3; ft = (aq + qpi) / hs - 0.5; }
                else { set_error("grid: edge face of panel %d edge %d t %d has no partner", p, e, t); return CSDYN_EINVAL; }
                F.t = int(std::lround(ft));
                if (std::fabs(ft - F.t) > 1e-8) { set_error("grid: non-conforming edge face"); return CSDYN_EINVAL; }
            }
    const size_t nf = this->nf();
    a11x.assign(nf, 0); a12x.assign(nf, 0); a22y.assign(nf, 0); a12y.assign(nf, 0); sc.assign(size_t(n) * n, 0);
    t1.assign(6 * nf * 3, 0); t2.assign(6 * nf * 3, 0); nrm.assign(6 * size_t(n) * n * 3, 0);
    gc1.assign(6 * size_t(n) * n * 3, 0); gc2.assign(6 * size_t(n) * n * 3, 0);
    rk.assign(nr, 0); rf.assign(nr + 1, 0); vol.assign(6 * size_t(nr) * n * n, 0);
    auto face_x = [&](int j, int fi, double &X, double &Y) { X = std::tan(-qpi + fi * hs); Y = std::tan(ang(j)); };
    auto face_y = [&](int fj, int i, double &X, double &Y) { X = std::tan(ang(i)); Y = std::tan(-qpi + fj * hs); };
    for (int j = 0; j < n; ++j)
        for (int fi = 0; fi <= n; ++fi) {
            double X, Y; face_x(j, fi, X, Y);
            double rho2 = 1 + X * X + Y * Y, rho = std::sqrt(rho2);
            size_t a = size_t(j) * (n + 1) + fi;
            a11x[a] = (1 + Y * Y) / rho;
            a12x[a] = X * Y / rho;
            double loc[3] = {-X * (1 + Y * Y) / rho2, (1 + Y * Y) / rho2, 0.0};
            for (int p = 0; p < 6; ++p) to_global(p, loc, &t1[(p * nf + a) * 3]);
        }
    for (int fj = 0; fj <= n; ++fj)
        for (int i = 0; i < n; ++i) {
            double X, Y; face_y(fj, i, X, Y);
            double rho2 = 1 + X * X + Y * Y, rho = std::sqrt(rho2);
            size_t a = size_t(fj) * n + i;
            a22y[a] = (1 + X * X) / rho;
            a12y[a] = X * Y / rho;
            double loc[3] = {-Y * (1 + X * X) / rho2, 0.0, (1 + X * X) / rho2};
            for (int p = 0; p < 6; ++p) to_global(p, loc, &t2[(p * nf + a) * 3]);
        }
    for (int j = 0; j < n; ++j)
        for (int i = 0; i < n; ++i) {
            double X = std::tan(ang(i)), Y = std::tan(ang(j));
            double rho2 = 1 + X * X + Y * Y, rho = std::sqrt(rho2);
            sc[size_t(j) * n + i] = (1 + X * X) * (1 + Y * Y) / (rho2 * rho);
            double loc[3] = {1.0 / rho, X / rho, Y / rho};
            double l1[3] = {-X * rho / (1 + X * X), rho / (1 + X * X), 0.0};
            double l2[3] = {-Y * rho / (1 + Y * Y), 0.0, rho / (1 + Y * Y)};
            for (int p = 0; p < 6; ++p) {
                const size_t a = ((size_t(p) * n + j) * n + i) * 3;
                to_global(p, loc, &nrm[a]);
                to_global(p, l1, &gc1[a]);
                to_global(p, l2, &gc2[a]);
            }
        }
    for (int k = 0; k < nr; ++k) rk[k] = rad(k);
    for (int k = 0; k <= nr; ++k) rf[k] = ri + k * hr;
    lay.assign(size_t(nr) * 8, 0.0);
    for (int k = 0; k < nr; ++k) {
        double *L = &lay[size_t(k) * 8];
        L[0] = rk[k];
        L[1] = 1.0 / (rk[k] * rk[k]);
        L[2] = rf[k] * rf[k];
        L[3] = rf[k + 1] * rf[k + 1];
        L[4] = 1.0 / (rk[k] * rk[k] * hr * hr);
        L[5] = 0.5 / (rk[k] * rk[k] * hr);
        L[6] = 1.0 / rk[k];
    }
    isc.assign(size_t(n) * n, 0.0);
    for (size_t a = 0; a < size_t(n) * n; ++a) isc[a] = 1.0 / (hs * sc[a]);
    for (int p = 0; p < 6; ++p)
        for (int k = 0; k < nr; ++k)
            for (int j = 0; j < n; ++j)
                for (int i = 0; i < n; ++i)
                    vol[cell(p, i, j, k)] = rk[k] * rk[k] * sc[size_t(j) * n + i] * hs * hs * hr;
    return CSDYN_OK;
}

size_t devgeom_bytes(int n, int nr) {
    Carver c(nullptr);
    size_t nf = size_t(n) * (n + 1);
    c.take<double>(nf); c.take<double>(nf); c.take<double>(nf); c.take<double>(nf);
    c.take<double>(size_t(n) * n);
    c.take<double>(6 * nf * 3); c.take<double>(6 * nf * 3); c.take<double>(6 * size_t(n) * n * 3);
    c.take<double>(6 * size_t(n) * n * 3); c.take<double>(6 * size_t(n) * n * 3);
    c.take<double>(nr); c.take<double>(nr + 1);
    c.take<double>(size_t(nr) * 8); c.take<double>(size_t(n) * n);
    c.take<int>(24 * size_t(n) * 4); c.take<double>(24 * size_t(n) * 4); c.take<int>(24 * size_t(n) * 4);
    c.take<double>(6 * size_t(nr) * n * n);
    c.take<double>(24 * size_t(nr) * n * 4);
    c.take<double>(24 * size_t(nr) * n * 8);
    c.take<double>(64);
    c.take<double>(2048);
    return c.off + 256;
}

int32_t devgeom_setup(const HostGeom &hg, void *ws, DevGeom *o) {
    const int n = hg.n, nr = hg.nr;
    const size_t nf = size_t(n) * (n + 1);
    Carver c(ws);
    o->n = n; o->nr = nr; o->hs = hg.hs; o->hr = hg.hr;
    o->a11x = c.take<double>(nf); o->a12x = c.take<double>(nf);
    o->a22y = c.take<double>(nf); o->a12y = c.take<double>(nf);
    o->sc = c.take<double>(size_t(n) * n);
    o->t1 = c.take<double>(6 * nf * 3); o->t2 = c.take<double>(6 * nf * 3);
    o->nrm = c.take<double>(6 * size_t(n) * n * 3);
    o->gc1 = c.take<double>(6 * size_t(n) * n * 3);
    o->gc2 = c.take<double>(6 * size_t(n) * n * 3);
    o->rk = c.take<double>(nr); o->rf = c.take<double>(nr + 1);
    o->lay = c.take<double>(size_t(nr) * 8); o->isc = c.take<double>(size_t(n) * n);
    {
        const double rbot = hg.rf[0] - 0.5 * hg.hr, rtop = hg.rf[nr] + 0.5 * hg.hr;
        o->wq2_bot = (hg.rk[0] / rbot) * (hg.rk[0] / rbot);
        o->wq2_top = (hg.rk[nr - 1] / rtop) * (hg.rk[nr - 1] / rtop);
    }
    o->gh_i = c.take<int>(24 * size_t(n) * 4); o->gh_w = c.take<double>(24 * size_t(n) * 4);
    o->fc = c.take<int>(24 * size_t(n) * 4);
    o->vol = c.take<double>(6 * size_t(nr) * n * n);
    o->G = c.take<double>(24 * size_t(nr) * n * 4);
    o->SF = c.take<double>(24 * size_t(nr) * n * 8);
    o->zero = c.take<double>(64);
    o->sink = c.take<double>(2048);
    CSD_HIP(hipMemset(o->zero, 0, 64 * sizeof(double)));

    std::vector<int> ghi(24 * size_t(n) * 4), fcv(24 * size_t(n) * 4);
    std::vector<double> ghw(24 * size_t(n) * 4);
    for (size_t a = 0; a < 24 * size_t(n); ++a) {
        const GhostEntry &G = hg.ghost[a];
        ghi[4 * a] = G.q; ghi[4 * a + 1] = G.fix_i; ghi[4 * a + 2] = G.idx; ghi[4 * a + 3] = G.m0;
        for (int m = 0; m < 4; ++m) ghw[4 * a + m] = G.w[m];
        const FaceEntry &F = hg.face[a];
        fcv[4 * a] = F.q; fcv[4 * a + 1] = F.e; fcv[4 * a + 2] = F.t; fcv[4 * a + 3] = 0;
    }
    const std::vector<double> &a11x = hg.a11x, &a12x = hg.a12x, &a22y = hg.a22y, &a12y = hg.a12y, &sc = hg.sc,
                              &t1 = hg.t1, &t2 = hg.t2, &nrm = hg.nrm, &rk = hg.rk, &rf = hg.rf, &vol = hg.vol,
                              &gc1 = hg.gc1, &gc2 = hg.gc2, &lay = hg.lay, &isc = hg.isc;
    auto up = [](void *dst, const void *src, size_t bytes) { return hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice); };
#define UP(dst, vec) CSD_HIP(up(dst, vec.data(), vec.size() * sizeof(vec[0])))
    UP(o->a11x, a11x); UP(o->a12x, a12x); UP(o->a22y, a22y); UP(o->a12y, a12y); UP(o->sc, sc);
    UP(o->t1, t1); UP(o->t2, t2); UP(o->nrm, nrm); UP(o->rk, rk); UP(o->rf, rf); UP(o->gc1, gc1); UP(o->gc2, gc2);
    UP(o->lay, lay); UP(o->isc, isc);
    UP(o->gh_i, ghi); UP(o->gh_w, ghw); UP(o->fc, fcv); UP(o->vol, vol);
#undef UP
    return CSDYN_OK;
}

}  // namespace csd
