/*
 * csdyn_ref.c -- plain FP64 CPU oracle for the cubed-sphere shell solver.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no code, header or table with the HIP
 * path: it re-derives every quantity from the paper's definitions, written
 * for clarity rather than speed.
 *
 * Paper: Yin, Yang, Ma, Cai, Zhang, "Parallel finite volume simulation of
 * the spherical shell dynamo with pseudo-vacuum magnetic boundary
 * conditions" (arXiv 2009.02171).
 *
 * What is computed (each function cites the passage it follows):
 *   - grid and metric of the equiangular gnomonic cubed-sphere shell
 *     (Sec. 3.2, cell-centre coordinates and the sqrt(g) formula);
 *   - the finite-volume divergence by Gauss' theorem (Sec. 3.2, eq.
 *     divdiscretization), used for the Laplacian (divergence of the
 *     gradient) and for D(v);
 *   - wall conditions: no-slip (eq. utb), Neumann pressure and Dirichlet
 *     pseudo-pressure (Sec. 3.1, after eq. tspb), pseudo-vacuum B
 *     (eq. pvc and the d(r^2 B^3)/dr = 0 relation of Sec. 3.2);
 *   - the two systems of the approximate factorization (Sec. 3.1), each as
 *     one 4-unknown-per-cell block lower-triangular system (readings below);
 *   - the one-level RAS preconditioner with ILU(0) subdomain solves
 *     (Sec. 3.3, eq. onelevel), the hybrid two-level preconditioner
 *     (eq. twolevel, coarsesolve, finesolve) and right-preconditioned
 *     restarted GMRES / flexible GMRES (Sec. 3.3, eq. newlinear and the
 *     stopping rule that follows it).
 *
 * Readings where the paper is silent (the predecessor paper that holds the
 * Laplacian and ghost-cell details is not available):
 *   R1 panels 0-3 are equatorial, centred on +x,+y,-x,-y, with xi eastward
 *      and eta northward; panel 4 is +z, panel 5 is -z; rotation axis +z.
 *   R2 unknowns are stored as Cartesian vector components plus a scalar;
 *      contravariant components appear only at faces.
 *   R3 the scalar Laplacian is the FV divergence of the face gradient
 *      sqrt(g) g^{mn} d_n f, with the cross derivative at a face taken as
 *      the mean of the two adjacent central differences (an 11-point
 *      stencil).  D(v) uses the face value (v_c + v_nb)/2.
 *   R4 ghost cells across a panel edge are cubic (4-point) Lagrange
 *      interpolants along the neighbour panel's first cell layer, in the
 *      neighbour's equiangular coordinate, shifted one-sided near edge ends;
 *      the cube-corner ghost is f(-1,0) + f(0,-1) - f(0,0).
 *   R5 a flux through a panel-edge face is the mean of the two panels'
 *      one-sided evaluations (so the scheme is exactly conservative).
 *   R6 wall ghosts: u_g = -u_in; P_g = P_in; P_b,g = -P_b,in; for B the
 *      tangential part flips sign and the radial part is scaled by
 *      (r_in/r_g)^2.
 *   R7 velocity-pressure (VP) rows: u - dt(E lap u - 2 zhat x u) and
 *      D(u) - dt lap_N P.  Magnetic (BP) rows: B - dt (E/Pm) lap B and
 *      D(B) - dt lap_D P_b.
 *   R8 subdomain matrices use the structural stencil pattern (every
 *      (row, col) pair the stencil expansion reaches, whatever its value)
 *      restricted to the overlapping box; rows are ordered box-
 *      lexicographically (i fastest, then j, then k), cell-major,
 *      component-minor.  ILU(0) is point-wise.
 *   R9 two-level: restriction is the mean of the 8 children, prolongation
 *      copies to the children, the coarse operator is re-discretised on the
 *      N/2, Nr/2 grid, the coarse solve is GMRES(30) with one-level RAS,
 *      x0 = 0, relative tolerance 0.1.  For the singular Neumann (VP)
 *      system the pressure part of a right-hand side is projected to zero
 *      volume-weighted mean before a solve.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <stdio.h>

#define REF_OK 0
#define REF_ENOTCONV 1
#define REF_EINVAL (-1)
#define REF_EZEROPIVOT (-3)
#define REF_ENOMEM (-4)
#define REF_EBREAKDOWN (-5)

typedef struct { int32_t n, nr; double ri, ro; } ref_grid;
typedef struct { int32_t kind; double dt, ekman, pm, ra, pr; } ref_op;   /* kind 0 = VP, 1 = BP, 2 = VT */

static const double QPI = 0.78539816339744830962; /* pi/4 */

/* ---------------------------------------------------------------- geometry */
/* Global Cartesian = PM[p] * (a, b, c) where (a, b, c) = (1, tan xi, tan eta)
 * up to normalisation (reading R1). */
static const int PM[6][3][3] = {
    {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}},
    {{0, -1, 0}, {1, 0, 0}, {0, 0, 1}},
    {{-1, 0, 0}, {0, -1, 0}, {0, 0, 1}},
    {{0, 1, 0}, {-1, 0, 0}, {0, 0, 1}},
    {{0, 0, -1}, {0, 1, 0}, {1, 0, 0}},
    {{0, 0, 1}, {0, 1, 0}, {-1, 0, 0}},
};

static double hs_of(const ref_grid *g) { return 2.0 * QPI / g->n; }
static double hr_of(const ref_grid *g) { return (g->ro - g->ri) / g->nr; }
static double xi_of(const ref_grid *g, double i) { return -QPI + (i + 0.5) * hs_of(g); }
static double r_of(const ref_grid *g, double k) { return g->ri + (k + 0.5) * hr_of(g); }

static void rot(int p, const double l[3], double out[3]) {
    for (int a = 0; a < 3; a++)
        out[a] = PM[p][a][0] * l[0] + PM[p][a][1] * l[1] + PM[p][a][2] * l[2];
}
static void rot_t(int p, const double v[3], double out[3]) {
    for (int a = 0; a < 3; a++)
        out[a] = PM[p][0][a] * v[0] + PM[p][1][a] * v[1] + PM[p][2][a] * v[2];
}

/* Covariant basis of x = r (1, X, Y)/rho, X = tan xi, Y = tan eta, by
 * differentiating the embedding; the contravariant basis is the inverse of
 * the Jacobian and sqrt(g) its determinant (Sec. 3.2). */
typedef struct { double sqrtg; double gcov[3][3]; double gcon[3][3]; } metric;

static void metric_at(int p, double xi, double eta, double r, metric *m) {
    double X = tan(xi), Y = tan(eta);
    double sx = 1.0 + X * X, sy = 1.0 + Y * Y; /* sec^2 */
    double rho2 = 1.0 + X * X + Y * Y, rho = sqrt(rho2), rho3 = rho2 * rho;
    double g1[3] = {-X, 1.0 + Y * Y, -X * Y}, g2[3] = {-Y, -X * Y, 1.0 + X * X}, g3[3] = {1.0, X, Y};
    double J[3][3]; /* columns are g_1, g_2, g_3 (local frame) */
    for (int a = 0; a < 3; a++) {
        J[a][0] = r * sx * g1[a] / rho3;
        J[a][1] = r * sy * g2[a] / rho3;
        J[a][2] = g3[a] / rho;
    }
    double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
               - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
               + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
    double inv[3][3]; /* inv = J^{-1}: rows are g^1, g^2, g^3 */
    inv[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
    inv[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
    inv[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
    inv[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
    inv[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
    inv[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
    inv[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
    inv[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
    inv[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
    m->sqrtg = det;
    for (int n = 0; n < 3; n++) {
        double col[3] = {J[0][n], J[1][n], J[2][n]};
        rot(p, col, m->gcov[n]);
        rot(p, inv[n], m->gcon[n]);
    }
}

static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* ------------------------------------------------------ panel-edge tables */
/* Edges: 0 = W (i = -1), 1 = E (i = N), 2 = S (j = -1), 3 = N (j = N). */
typedef struct {
    int q;         /* neighbour panel holding the ghost point */
    int fix_i;     /* 1: the interpolation line has fixed i (= idx), varying j */
    int idx;       /* fixed index (0 or N-1) */
    int m0;        /* first of the 4 nodes along the line */
    double w[4];   /* Lagrange weights */
} ghost_info;

typedef struct { int q, eq, tq; } face_info; /* matching face on panel q */

typedef struct {
    ref_grid g;
    ghost_info *gh; /* [6][4][N] */
    face_info *fc;  /* [6][4][N] */
} seam_tab;

static void edge_point(const ref_grid *g, int e, int t, int ghost, double *xi, double *eta) {
    double off = ghost ? -1.0 : -0.5;   /* ghost centre, or face centre */
    double lo = off, hi = g->n - 1 - off;
    switch (e) {
    case 0: *xi = xi_of(g, lo); *eta = xi_of(g, t); break;
    case 1: *xi = xi_of(g, hi); *eta = xi_of(g, t); break;
    case 2: *xi = xi_of(g, t); *eta = xi_of(g, lo); break;
    default: *xi = xi_of(g, t); *eta = xi_of(g, hi); break;
    }
}

static void to_panel(int q, const double d[3], double *xi, double *eta, double *a) {
    double l[3];
    rot_t(q, d, l);
    *a = l[0];
    *xi = atan(l[1] / l[0]);
    *eta = atan(l[2] / l[0]);
}

static int build_seams(const ref_grid *g, seam_tab *st) {
    int n = g->n;
    double h = hs_of(g);
    st->g = *g;
    st->gh = calloc((size_t)24 * n, sizeof(ghost_info));
    st->fc = calloc((size_t)24 * n, sizeof(face_info));
    if (!st->gh || !st->fc) return REF_ENOMEM;
    for (int p = 0; p < 6; p++)
        for (int e = 0; e < 4; e++)
            for (int t = 0; t < n; t++) {
                double xi, eta, d[3], l[3];
                edge_point(g, e, t, 1, &xi, &eta);
                l[0] = 1.0; l[1] = tan(xi); l[2] = tan(eta);
                rot(p, l, d);
                int best = -1; double ba = -1e300;
                for (int q = 0; q < 6; q++) {
                    double lq[3]; rot_t(q, d, lq);
                    if (lq[0] > ba) { ba = lq[0]; best = q; }
                }
                double xq, eq, aq;
                to_panel(best, d, &xq, &eq, &aq);
                double fi = (xq + QPI) / h - 0.5, fj = (eq + QPI) / h - 0.5;
                ghost_info *gi = &st->gh[(p * 4 + e) * n + t];
                gi->q = best;
                double s;
                if (fabs(xq) > fabs(eq)) { gi->fix_i = 1; gi->idx = (int)lround(fi); s = fj; if (fabs(fi - gi->idx) > 1e-8) return REF_EINVAL; }
                else { gi->fix_i = 0; gi->idx = (int)lround(fj); s = fi; if (fabs(fj - gi->idx) > 1e-8) return REF_EINVAL; }
                if (gi->idx != 0 && gi->idx != n - 1) return REF_EINVAL;
                int m0 = (int)floor(s) - 1;
                if (m0 < 0) m0 = 0;
                if (m0 > n - 4) m0 = n - 4;
                gi->m0 = m0;
                for (int m = 0; m < 4; m++) {
                    double w = 1.0;
                    for (int l2 = 0; l2 < 4; l2++)
                        if (l2 != m) w *= (s - (m0 + l2)) / (double)(m - l2);
                    gi->w[m] = w;
                }
                /* matching face */
                edge_point(g, e, t, 0, &xi, &eta);
                l[0] = 1.0; l[1] = tan(xi); l[2] = tan(eta);
                rot(p, l, d);
                to_panel(best, d, &xq, &eq, &aq);
                face_info *fi2 = &st->fc[(p * 4 + e) * n + t];
                fi2->q = best;
                double tq;
                if (fabs(fabs(xq) - QPI) < 1e-12) { fi2->eq = xq < 0 ? 0 : 1; tq = (eq + QPI) / h - 0.5; }
                else if (fabs(fabs(eq) - QPI) < 1e-12) { fi2->eq = eq < 0 ? 2 : 3; tq = (xq + QPI) / h - 0.5; }
                else return REF_EINVAL;
                fi2->tq = (int)lround(tq);
                if (fabs(tq - fi2->tq) > 1e-8) return REF_EINVAL;
            }
    return REF_OK;
}

static void free_seams(seam_tab *st) { free(st->gh); free(st->fc); st->gh = NULL; st->fc = NULL; }

/* ------------------------------------------------------------ term sinks */
typedef struct { int64_t col; double w; } term;
typedef struct {
    term *t; size_t n, cap;
    const double *x; double acc; int mode; /* mode 0: collect terms, 1: accumulate w*x[col] */
} sink;

static void sink_add(sink *s, int64_t col, double w) {
    if (s->mode == 1) { s->acc += w * s->x[col]; return; }
    if (s->n == s->cap) {
        s->cap = s->cap ? 2 * s->cap : 256;
        s->t = realloc(s->t, s->cap * sizeof(term));
    }
    s->t[s->n].col = col; s->t[s->n].w = w; s->n++;
}

typedef struct {
    ref_grid g; ref_op op; const seam_tab *st;
} ctx;

static int64_t unk(const ref_grid *g, int p, int i, int j, int k, int c) {
    return ((((int64_t)p * g->nr + k) * g->n + j) * g->n + i) * 4 + c;
}

static void unit_radial(const ref_grid *g, int p, int i, int j, double n[3]) {
    double l[3] = {1.0, tan(xi_of(g, i)), tan(xi_of(g, j))};
    double rho = sqrt(dot3(l, l));
    for (int a = 0; a < 3; a++) l[a] /= rho;
    rot(p, l, n);
}

/* Value of component c at the extended position (p,i,j,k): a real unknown,
 * or a ghost expressed through real unknowns (readings R4, R6). */
static void emit_x(const ctx *cx, sink *s, int p, int i, int j, int k, int c, double w) {
    const ref_grid *g = &cx->g;
    int n = g->n;
    if (k < 0 || k >= g->nr) {
        int kin = k < 0 ? 0 : g->nr - 1;
        if (cx->op.kind == 0) {
            emit_x(cx, s, p, i, j, kin, c, c < 3 ? -w : w);
        } else if (cx->op.kind == 2) {   /* no-slip u, isothermal Theta = 0 */
            emit_x(cx, s, p, i, j, kin, c, -w);
        } else {
            if (c < 3) {
                double nr[3]; unit_radial(g, p, i, j, nr);
                double q = r_of(g, kin) / r_of(g, k); q = q * q;
                for (int d = 0; d < 3; d++)
                    emit_x(cx, s, p, i, j, kin, d, w * ((c == d ? -1.0 : 0.0) + (1.0 + q) * nr[c] * nr[d]));
            } else {
                emit_x(cx, s, p, i, j, kin, 3, -w);
            }
        }
        return;
    }
    int iin = i >= 0 && i < n, jin = j >= 0 && j < n;
    if (iin && jin) { sink_add(s, unk(g, p, i, j, k, c), w); return; }
    if (!iin && !jin) { /* cube corner */
        int ic = i < 0 ? 0 : n - 1, jc = j < 0 ? 0 : n - 1;
        emit_x(cx, s, p, i, jc, k, c, w);
        emit_x(cx, s, p, ic, j, k, c, w);
        emit_x(cx, s, p, ic, jc, k, c, -w);
        return;
    }
    int e, t;
    if (!iin) { e = i < 0 ? 0 : 1; t = j; } else { e = j < 0 ? 2 : 3; t = i; }
    const ghost_info *gi = &cx->st->gh[(p * 4 + e) * n + t];
    for (int m = 0; m < 4; m++) {
        int a = gi->m0 + m;
        if (gi->fix_i) emit_x(cx, s, gi->q, gi->idx, a, k, c, w * gi->w[m]);
        else emit_x(cx, s, gi->q, a, gi->idx, k, c, w * gi->w[m]);
    }
}

/* One-sided outward Laplacian flux sqrt(g) g^{mn} d_n f through a lateral
 * face of cell (i,j,k) of panel p, evaluated with panel p's own (extended)
 * values (reading R3).  face: 0 W, 1 E, 2 S, 3 N. */
static void emit_lat_lap_flux(const ctx *cx, sink *s, int p, int i, int j, int k, int face, int c, double w) {
    const ref_grid *g = &cx->g;
    double h = hs_of(g), r = r_of(g, k);
    metric m;
    if (face <= 1) {
        int il = face == 0 ? i - 1 : i, ir = il + 1;   /* face between il and ir */
        metric_at(p, -QPI + (ir) * h, xi_of(g, j), r, &m);
        double a11 = m.sqrtg * dot3(m.gcon[0], m.gcon[0]);
        double a12 = m.sqrtg * dot3(m.gcon[0], m.gcon[1]);
        double sg = face == 1 ? w : -w;      /* +F for E, -F for W */
        emit_x(cx, s, p, ir, j, k, c, sg * a11 / h);
        emit_x(cx, s, p, il, j, k, c, -sg * a11 / h);
        double q = sg * a12 / (4.0 * h);
        emit_x(cx, s, p, il, j + 1, k, c, q);
        emit_x(cx, s, p, ir, j + 1, k, c, q);
        emit_x(cx, s, p, il, j - 1, k, c, -q);
        emit_x(cx, s, p, ir, j - 1, k, c, -q);
    } else {
        int jl = face == 2 ? j - 1 : j, jr = jl + 1;
        metric_at(p, xi_of(g, i), -QPI + (jr) * h, r, &m);
        double a22 = m.sqrtg * dot3(m.gcon[1], m.gcon[1]);
        double a12 = m.sqrtg * dot3(m.gcon[0], m.gcon[1]);
        double sg = face == 3 ? w : -w;
        emit_x(cx, s, p, i, jr, k, c, sg * a22 / h);
        emit_x(cx, s, p, i, jl, k, c, -sg * a22 / h);
        double q = sg * a12 / (4.0 * h);
        emit_x(cx, s, p, i + 1, jl, k, c, q);
        emit_x(cx, s, p, i + 1, jr, k, c, q);
        emit_x(cx, s, p, i - 1, jl, k, c, -q);
        emit_x(cx, s, p, i - 1, jr, k, c, -q);
    }
}

/* One-sided outward flux of sqrt(g) g^m . v through a lateral face, with the
 * face value (v_c + v_nb)/2 (reading R3). */
static void emit_lat_div_flux(const ctx *cx, sink *s, int p, int i, int j, int k, int face, double w) {
    const ref_grid *g = &cx->g;
    double h = hs_of(g), r = r_of(g, k);
    metric m;
    int ni = i, nj = j, mm;
    if (face <= 1) { ni = face == 0 ? i - 1 : i + 1; mm = 0; metric_at(p, -QPI + (face == 0 ? i : i + 1) * h, xi_of(g, j), r, &m); }
    else { nj = face == 2 ? j - 1 : j + 1; mm = 1; metric_at(p, xi_of(g, i), -QPI + (face == 2 ? j : j + 1) * h, r, &m); }
    double sg = (face == 1 || face == 3) ? w : -w;
    for (int d = 0; d < 3; d++) {
        double cf = sg * m.sqrtg * m.gcon[mm][d] * 0.5;
        emit_x(cx, s, p, i, j, k, d, cf);
        emit_x(cx, s, p, ni, nj, k, d, cf);
    }
}

static int is_seam_face(const ref_grid *g, int i, int j, int face) {
    return (face == 0 && i == 0) || (face == 1 && i == g->n - 1) || (face == 2 && j == 0) || (face == 3 && j == g->n - 1);
}

/* First-layer cell of panel q adjacent to its edge eq at tangential index t. */
static void edge_cell(const ref_grid *g, int eq, int t, int *i, int *j) {
    switch (eq) {
    case 0: *i = 0; *j = t; break;
    case 1: *i = g->n - 1; *j = t; break;
    case 2: *i = t; *j = 0; break;
    default: *i = t; *j = g->n - 1; break;
    }
}

/* w * (finite-volume Laplacian of component c) at cell (p,i,j,k):
 * (1/V) * sum over faces of outward flux * face area, V = sqrt(g)_c hs^2 hr
 * (eq. divdiscretization applied to the gradient; readings R3-R6). */
static void emit_laplacian(const ctx *cx, sink *s, int p, int i, int j, int k, int c, double w) {
    const ref_grid *g = &cx->g;
    double h = hs_of(g), hr = hr_of(g);
    metric mc; metric_at(p, xi_of(g, i), xi_of(g, j), r_of(g, k), &mc);
    double V = mc.sqrtg * h * h * hr;
    double wl = w * h * hr / V, wr = w * h * h / V;
    for (int f = 0; f < 4; f++) {
        if (!is_seam_face(g, i, j, f)) { emit_lat_lap_flux(cx, s, p, i, j, k, f, c, wl); continue; }
        int t = f <= 1 ? j : i;
        const face_info *fi = &cx->st->fc[(p * 4 + f) * g->n + t];
        int iq, jq; edge_cell(g, fi->eq, fi->tq, &iq, &jq);
        emit_lat_lap_flux(cx, s, p, i, j, k, f, c, 0.5 * wl);
        emit_lat_lap_flux(cx, s, fi->q, iq, jq, k, fi->eq, c, -0.5 * wl);
    }
    /* radial faces: sqrt(g) at r_{k+-1/2}, g^33 = 1 */
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        metric mf; metric_at(p, xi_of(g, i), xi_of(g, j), r_of(g, k + 0.5 * sgn), &mf);
        double cf = wr * mf.sqrtg * dot3(mf.gcon[2], mf.gcon[2]) / hr;
        emit_x(cx, s, p, i, j, k + sgn, c, cf);
        emit_x(cx, s, p, i, j, k, c, -cf);
    }
}

/* w * D(v) at cell (p,i,j,k) with v the Cartesian components 0..2. */
static void emit_divergence(const ctx *cx, sink *s, int p, int i, int j, int k, double w) {
    const ref_grid *g = &cx->g;
    double h = hs_of(g), hr = hr_of(g);
    metric mc; metric_at(p, xi_of(g, i), xi_of(g, j), r_of(g, k), &mc);
    double V = mc.sqrtg * h * h * hr;
    double wl = w * h * hr / V, wr = w * h * h / V;
    for (int f = 0; f < 4; f++) {
        if (!is_seam_face(g, i, j, f)) { emit_lat_div_flux(cx, s, p, i, j, k, f, wl); continue; }
        int t = f <= 1 ? j : i;
        const face_info *fi = &cx->st->fc[(p * 4 + f) * g->n + t];
        int iq, jq; edge_cell(g, fi->eq, fi->tq, &iq, &jq);
        emit_lat_div_flux(cx, s, p, i, j, k, f, 0.5 * wl);
        emit_lat_div_flux(cx, s, fi->q, iq, jq, k, fi->eq, -0.5 * wl);
    }
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        metric mf; metric_at(p, xi_of(g, i), xi_of(g, j), r_of(g, k + 0.5 * sgn), &mf);
        for (int d = 0; d < 3; d++) {
            double cf = sgn * wr * mf.sqrtg * mf.gcon[2][d] * 0.5;
            emit_x(cx, s, p, i, j, k, d, cf);
            emit_x(cx, s, p, i, j, k + sgn, d, cf);
        }
    }
}

/* One row of the system matrix (reading R7; Sec. 3.1).  Kind 2 (VT) is the
 * velocity-temperature block of the VTBE (eq. tsvelocity, tstemperature) in
 * the same scaling, Delta t / 2 = E dt: u rows with -(Delta t/2) R1(Theta) =
 * -dt Ra/r_o Theta x, Theta row Theta - dt (E/Pr) lap Theta - (Delta t/2)
 * R2(u) with R2(u) = r_i r_o / r^3 (x . u) (eq. linearoperator). */
static void emit_row(const ctx *cx, sink *s, int p, int i, int j, int k, int c) {
    double dt = cx->op.dt, E = cx->op.ekman;
    if (cx->op.kind == 2) {
        const ref_grid *g = &cx->g;
        double nr3[3]; unit_radial(g, p, i, j, nr3);
        double r = r_of(g, k);
        if (c < 3) {
            emit_x(cx, s, p, i, j, k, c, 1.0);
            emit_laplacian(cx, s, p, i, j, k, c, -dt * E);
            if (c == 0) emit_x(cx, s, p, i, j, k, 1, -2.0 * dt);
            if (c == 1) emit_x(cx, s, p, i, j, k, 0, 2.0 * dt);
            emit_x(cx, s, p, i, j, k, 3, -dt * cx->op.ra / g->ro * r * nr3[c]);
        } else {
            emit_x(cx, s, p, i, j, k, 3, 1.0);
            emit_laplacian(cx, s, p, i, j, k, 3, -dt * E / cx->op.pr);
            for (int d = 0; d < 3; d++)
                emit_x(cx, s, p, i, j, k, d, -dt * E * g->ri * g->ro / (r * r * r) * r * nr3[d]);
        }
        return;
    }
    if (cx->op.kind == 0) {
        if (c < 3) {
            emit_x(cx, s, p, i, j, k, c, 1.0);
            emit_laplacian(cx, s, p, i, j, k, c, -dt * E);
            if (c == 0) emit_x(cx, s, p, i, j, k, 1, -2.0 * dt);   /* +2dt (zhat x u)_x = -2dt u_y */
            if (c == 1) emit_x(cx, s, p, i, j, k, 0, 2.0 * dt);    /* +2dt (zhat x u)_y = +2dt u_x */
        } else {
            emit_divergence(cx, s, p, i, j, k, 1.0);
            emit_laplacian(cx, s, p, i, j, k, 3, -dt);
        }
    } else {
        if (c < 3) {
            emit_x(cx, s, p, i, j, k, c, 1.0);
            emit_laplacian(cx, s, p, i, j, k, c, -dt * E / cx->op.pm);
        } else {
            emit_divergence(cx, s, p, i, j, k, 1.0);
            emit_laplacian(cx, s, p, i, j, k, 3, -dt);
        }
    }
}

static int check_grid(const ref_grid *g) {
    if (!g || g->n < 4 || g->nr < 1 || !(g->ro > g->ri) || !(g->ri > 0)) return REF_EINVAL;
    return REF_OK;
}

/* ------------------------------------------------------ exported: geometry */
int ref_cell_geometry(const ref_grid *g, double *xyz, double *vol) {
    if (check_grid(g)) return REF_EINVAL;
    int n = g->n;
    double h = hs_of(g), hr = hr_of(g);
    for (int p = 0; p < 6; p++)
        for (int k = 0; k < g->nr; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    int64_t c = (((int64_t)p * g->nr + k) * n + j) * n + i;
                    double nr[3]; unit_radial(g, p, i, j, nr);
                    double r = r_of(g, k);
                    if (xyz) for (int a = 0; a < 3; a++) xyz[3 * c + a] = r * nr[a];
                    if (vol) { metric m; metric_at(p, xi_of(g, i), xi_of(g, j), r, &m); vol[c] = m.sqrtg * h * h * hr; }
                }
    return REF_OK;
}

/* Metric at an arbitrary point (for the geometry tests). */
int ref_metric(int p, double xi, double eta, double r, double *sqrtg, double *gcov9, double *gcon9) {
    metric m; metric_at(p, xi, eta, r, &m);
    *sqrtg = m.sqrtg;
    for (int a = 0; a < 3; a++) for (int b = 0; b < 3; b++) { gcov9[3 * a + b] = m.gcov[a][b]; gcon9[3 * a + b] = m.gcon[a][b]; }
    return REF_OK;
}

/* Seam tables (for the geometry tests): per (p, edge, t) the ghost's panel,
 * line, nodes and weights, and the matching face. */
int ref_seam_tables(const ref_grid *g, int32_t *gq, int32_t *gfix, int32_t *gidx, int32_t *gm0, double *gw,
                    int32_t *fq, int32_t *feq, int32_t *ftq) {
    if (check_grid(g)) return REF_EINVAL;
    seam_tab st; int rc = build_seams(g, &st);
    if (rc) { free_seams(&st); return rc; }
    for (int a = 0; a < 24 * g->n; a++) {
        gq[a] = st.gh[a].q; gfix[a] = st.gh[a].fix_i; gidx[a] = st.gh[a].idx; gm0[a] = st.gh[a].m0;
        for (int m = 0; m < 4; m++) gw[4 * a + m] = st.gh[a].w[m];
        fq[a] = st.fc[a].q; feq[a] = st.fc[a].eq; ftq[a] = st.fc[a].tq;
    }
    free_seams(&st);
    return REF_OK;
}

/* ------------------------------------------------------ exported: operator */
static int make_ctx(const ref_grid *g, const ref_op *op, seam_tab *st, ctx *cx) {
    if (check_grid(g) || !op || op->kind < 0 || op->kind > 2 || (op->kind == 2 && !(op->pr > 0))) return REF_EINVAL;
    int rc = build_seams(g, st);
    if (rc) { free_seams(st); return rc; }
    cx->g = *g; cx->op = *op; cx->st = st;
    return REF_OK;
}

/* y = A x, row by row from the stencil definition. */
int ref_operator_apply(const ref_grid *g, const ref_op *op, const double *x, double *y) {
    seam_tab st; ctx cx;
    int rc = make_ctx(g, op, &st, &cx);
    if (rc) return rc;
    sink s = {0}; s.mode = 1; s.x = x;
    int n = g->n;
    for (int p = 0; p < 6; p++)
        for (int k = 0; k < g->nr; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++)
                    for (int c = 0; c < 4; c++) {
                        s.acc = 0.0;
                        emit_row(&cx, &s, p, i, j, k, c);
                        y[unk(g, p, i, j, k, c)] = s.acc;
                    }
    free_seams(&st);
    return REF_OK;
}

/* y at selected rows only (sampled checks at full size). */
int ref_operator_rows(const ref_grid *g, const ref_op *op, const double *x, int64_t nrows, const int64_t *rows, double *y) {
    seam_tab st; ctx cx;
    int rc = make_ctx(g, op, &st, &cx);
    if (rc) return rc;
    sink s = {0}; s.mode = 1; s.x = x;
    int n = g->n;
    for (int64_t a = 0; a < nrows; a++) {
        int64_t r = rows[a];
        int c = (int)(r % 4); int64_t cell = r / 4;
        int i = (int)(cell % n); cell /= n;
        int j = (int)(cell % n); cell /= n;
        int k = (int)(cell % g->nr); int p = (int)(cell / g->nr);
        s.acc = 0.0;
        emit_row(&cx, &s, p, i, j, k, c);
        y[a] = s.acc;
    }
    free_seams(&st);
    return REF_OK;
}

/* ------------------------------------------------ exported: nonlinear terms */
/* Value of component c of field x at an extended position, with the ghost
 * rules of the context's system (readings R4, R6). */
static double val_ext(const ctx *cx, const double *x, int p, int i, int j, int k, int c) {
    sink s = {0};
    s.mode = 1; s.x = x; s.acc = 0.0;
    emit_x(cx, &s, p, i, j, k, c, 1.0);
    return s.acc;
}

/* One-sided outward advective flux through lateral face `face` of cell
 * (p,i,j,k), from panel p's own extended values: (a_f . sqrt(g) g^m) b_f,
 * with a_f and b_f the means of the cell's and its face neighbour's values
 * (eq. nonlinearint with the face values of reading R3); out[c], c < 3. */
static void adv_lat_flux(const ctx *ca, const double *a, const ctx *cb, const double *b, int p, int i, int j, int k,
                         int face, double out[4]) {
    const ref_grid *g = &ca->g;
    double h = hs_of(g), r = r_of(g, k);
    metric m;
    int ni = i, nj = j, mm;
    if (face <= 1) { ni = face == 0 ? i - 1 : i + 1; mm = 0; metric_at(p, -QPI + (face == 0 ? i : i + 1) * h, xi_of(g, j), r, &m); }
    else { nj = face == 2 ? j - 1 : j + 1; mm = 1; metric_at(p, xi_of(g, i), -QPI + (face == 2 ? j : j + 1) * h, r, &m); }
    double sg = (face == 1 || face == 3) ? 1.0 : -1.0;
    double af = 0.0;
    for (int d = 0; d < 3; d++)
        af += m.sqrtg * m.gcon[mm][d] * 0.5 * (val_ext(ca, a, p, i, j, k, d) + val_ext(ca, a, p, ni, nj, k, d));
    for (int c = 0; c < 4; c++)
        out[c] = sg * af * 0.5 * (val_ext(cb, b, p, i, j, k, c) + val_ext(cb, b, p, ni, nj, k, c));
}

/* (a . grad) b at cell (p,i,j,k) in the conservative form div(a b_c) of each
 * Cartesian component c (Sec. 3.2, eq. nonlinearint; with Cartesian
 * components the Christoffel source terms of the contravariant form vanish):
 * (1/V) * sum over the six faces of the outward flux times the face area,
 * the flux through a panel-edge face being the mean of the two panels'
 * one-sided fluxes (reading R5). */
static void adv_cell(const ctx *ca, const double *a, const ctx *cb, const double *b, int p, int i, int j, int k,
                     double out[4]) {
    const ref_grid *g = &ca->g;
    double h = hs_of(g), hr = hr_of(g);
    metric mc; metric_at(p, xi_of(g, i), xi_of(g, j), r_of(g, k), &mc);
    double V = mc.sqrtg * h * h * hr;
    double wl = h * hr / V, wr = h * h / V;
    double acc[4] = {0.0, 0.0, 0.0, 0.0}, f1[4], f2[4];
    for (int f = 0; f < 4; f++) {
        if (!is_seam_face(g, i, j, f)) {
            adv_lat_flux(ca, a, cb, b, p, i, j, k, f, f1);
            for (int c = 0; c < 4; c++) acc[c] += wl * f1[c];
            continue;
        }
        int t = f <= 1 ? j : i;
        const face_info *fi = &ca->st->fc[(p * 4 + f) * g->n + t];
        int iq, jq; edge_cell(g, fi->eq, fi->tq, &iq, &jq);
        adv_lat_flux(ca, a, cb, b, p, i, j, k, f, f1);
        adv_lat_flux(ca, a, cb, b, fi->q, iq, jq, k, fi->eq, f2);
        for (int c = 0; c < 4; c++) acc[c] += wl * 0.5 * (f1[c] - f2[c]);
    }
    for (int sgn = -1; sgn <= 1; sgn += 2) {
        metric mf; metric_at(p, xi_of(g, i), xi_of(g, j), r_of(g, k + 0.5 * sgn), &mf);
        double af = 0.0;
        for (int d = 0; d < 3; d++)
            af += mf.sqrtg * mf.gcon[2][d] * 0.5 * (val_ext(ca, a, p, i, j, k, d) + val_ext(ca, a, p, i, j, k + sgn, d));
        for (int c = 0; c < 4; c++)
            acc[c] += wr * sgn * af * 0.5 * (val_ext(cb, b, p, i, j, k, c) + val_ext(cb, b, p, i, j, k + sgn, c));
    }
    for (int c = 0; c < 4; c++) out[c] = acc[c];
}

/* out = (a . grad) b on every cell.  a takes the ghost rules of system
 * kind_a, b those of kind_b (0: no-slip velocity, 1: pseudo-vacuum magnetic
 * field, 2: no-slip velocity and isothermal Theta).  scalar = 0: the vector
 * part of b (components 0..2; component 3 of out is 0); scalar = 1: the
 * scalar part (component 3; components 0..2 of out are 0). */
int ref_advect(const ref_grid *g, int32_t kind_a, const double *a, int32_t kind_b, const double *b, int32_t scalar,
               double *out) {
    ref_op oa = {kind_a, 0.0, 0.0, 1.0, 0.0, 1.0}, ob = {kind_b, 0.0, 0.0, 1.0, 0.0, 1.0};
    seam_tab sa, sb; ctx ca, cb;
    int rc = make_ctx(g, &oa, &sa, &ca);
    if (rc) return rc;
    rc = make_ctx(g, &ob, &sb, &cb);
    if (rc) { free_seams(&sa); return rc; }
    int n = g->n;
    for (int p = 0; p < 6; p++)
        for (int k = 0; k < g->nr; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    double v[4];
                    adv_cell(&ca, a, &cb, b, p, i, j, k, v);
                    for (int c = 0; c < 4; c++) out[unk(g, p, i, j, k, c)] = (c == 3) == (scalar != 0) ? v[c] : 0.0;
                }
    free_seams(&sa);
    free_seams(&sb);
    return REF_OK;
}

static int cmp_term(const void *a, const void *b) {
    int64_t x = ((const term *)a)->col, y = ((const term *)b)->col;
    return x < y ? -1 : x > y;
}

/* Sort terms by column and merge duplicates (summing); keeps entries whose
 * sum is zero, so the pattern is structural (reading R8). */
static size_t merge_terms(term *t, size_t n) {
    qsort(t, n, sizeof(term), cmp_term);
    size_t o = 0;
    for (size_t a = 0; a < n; a++) {
        if (o > 0 && t[o - 1].col == t[a].col) t[o - 1].w += t[a].w;
        else t[o++] = t[a];
    }
    return o;
}

/* Global CSR of A.  Call with col = val = NULL to get nnz in rowptr[nrows]. */
int ref_assemble(const ref_grid *g, const ref_op *op, int64_t *rowptr, int32_t *col, double *val) {
    seam_tab st; ctx cx;
    int rc = make_ctx(g, op, &st, &cx);
    if (rc) return rc;
    sink s = {0};
    int n = g->n;
    int64_t nnz = 0;
    rowptr[0] = 0;
    for (int p = 0; p < 6; p++)
        for (int k = 0; k < g->nr; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++)
                    for (int c = 0; c < 4; c++) {
                        s.n = 0;
                        emit_row(&cx, &s, p, i, j, k, c);
                        size_t m = merge_terms(s.t, s.n);
                        int64_t r = unk(g, p, i, j, k, c);
                        if (col) for (size_t a = 0; a < m; a++) { col[nnz + a] = (int32_t)s.t[a].col; val[nnz + a] = s.t[a].w; }
                        nnz += m;
                        rowptr[r + 1] = nnz;
                    }
    free(s.t);
    free_seams(&st);
    return REF_OK;
}

/* ------------------------------------------------------------ subdomains */
typedef struct {
    int nloc;            /* local cells */
    int64_t *gcell;      /* [nloc] global cell index of each local cell */
    int *owned;          /* [nloc] 1 if the cell is in the non-overlapping part */
    /* local CSR over 4*nloc rows */
    int64_t *rp; int32_t *ci; double *v;
    int64_t *diag;       /* position of the diagonal in each row */
} subdomain;

typedef struct {
    ref_grid g; ref_op op;
    int sub[3], nb[3], overlap, nsd;
    subdomain *sd;
    int precision;       /* 0 FP64, 1 FP32 emulation */
} onelevel;

/* Global cell reached from owned-box position (p, i, j, k) by one step
 * across a panel edge; -1 if the position does not exist (cube corner,
 * beyond a wall).  Reading R8: the overlap layer across an edge is the
 * neighbour panel's first-layer cells adjacent to the box's edge faces. */
static int64_t box_cell(const ctx *cx, int p, int i, int j, int k) {
    const ref_grid *g = &cx->g;
    int n = g->n;
    if (k < 0 || k >= g->nr) return -1;
    int iin = i >= 0 && i < n, jin = j >= 0 && j < n;
    if (iin && jin) return (((int64_t)p * g->nr + k) * n + j) * n + i;
    if (!iin && !jin) return -1;
    int e, t;
    if (!iin) { e = i < 0 ? 0 : 1; t = j; } else { e = j < 0 ? 2 : 3; t = i; }
    const face_info *fi = &cx->st->fc[(p * 4 + e) * n + t];
    int iq, jq; edge_cell(g, fi->eq, fi->tq, &iq, &jq);
    return (((int64_t)fi->q * g->nr + k) * n + jq) * n + iq;
}

static void free_onelevel(onelevel *ol) {
    if (!ol) return;
    for (int s = 0; s < ol->nsd; s++) {
        subdomain *d = &ol->sd[s];
        free(d->gcell); free(d->owned); free(d->rp); free(d->ci); free(d->v); free(d->diag);
    }
    free(ol->sd);
    free(ol);
}

/* ILU(0) in place on a CSR matrix with sorted columns (Saad's IKJ form):
 * for each row i, for each k < i in the row: a_ik /= a_kk, then
 * a_ij -= a_ik a_kj for every j > k that is in row i's pattern.
 * (Sec. 3.3: ILU with no fill-in as the subdomain solver.) */
static int ilu0(int64_t nrow, const int64_t *rp, const int32_t *ci, double *v, int64_t *diag) {
    int64_t *pos = malloc(sizeof(int64_t) * (size_t)(nrow > 0 ? nrow : 1));
    if (!pos) return REF_ENOMEM;
    for (int64_t a = 0; a < nrow; a++) pos[a] = -1;
    for (int64_t i = 0; i < nrow; i++) {
        diag[i] = -1;
        for (int64_t q = rp[i]; q < rp[i + 1]; q++) { pos[ci[q]] = q; if (ci[q] == i) diag[i] = q; }
        if (diag[i] < 0) { free(pos); return REF_EZEROPIVOT; }
        for (int64_t q = rp[i]; q < rp[i + 1] && ci[q] < i; q++) {
            int64_t k = ci[q];
            v[q] /= v[diag[k]];
            for (int64_t u = diag[k] + 1; u < rp[k + 1]; u++) {
                int64_t pj = pos[ci[u]];
                if (pj >= 0) v[pj] -= v[q] * v[u];
            }
        }
        for (int64_t q = rp[i]; q < rp[i + 1]; q++) pos[ci[q]] = -1;
        if (!(fabs(v[diag[i]]) >= 1e-300)) { free(pos); return REF_EZEROPIVOT; }
    }
    free(pos);
    return REF_OK;
}

/* Build the overlapping subdomain s: box cells, the restriction of A to them
 * (A_i^delta = R_i A R_i^T, Sec. 3.3), and its ILU(0). */
static int build_subdomain(const ctx *cx, onelevel *ol, int s, int32_t *g2l) {
    const ref_grid *g = &cx->g;
    int n = g->n;
    int bi = s % ol->nb[0], bj = (s / ol->nb[0]) % ol->nb[1], bk = (s / (ol->nb[0] * ol->nb[1])) % ol->nb[2];
    int p = s / (ol->nb[0] * ol->nb[1] * ol->nb[2]);
    int d = ol->overlap;
    int i0 = bi * ol->sub[0] - d, i1 = (bi + 1) * ol->sub[0] + d;
    int j0 = bj * ol->sub[1] - d, j1 = (bj + 1) * ol->sub[1] + d;
    int k0 = bk * ol->sub[2] - d, k1 = (bk + 1) * ol->sub[2] + d;
    subdomain *sd = &ol->sd[s];
    size_t cap = (size_t)(i1 - i0) * (j1 - j0) * (k1 - k0);
    sd->gcell = malloc(sizeof(int64_t) * cap);
    sd->owned = malloc(sizeof(int) * cap);
    if (!sd->gcell || !sd->owned) return REF_ENOMEM;
    int nloc = 0;
    for (int k = k0; k < k1; k++)
        for (int j = j0; j < j1; j++)
            for (int i = i0; i < i1; i++) {
                int64_t gc = box_cell(cx, p, i, j, k);
                if (gc < 0) continue;
                sd->gcell[nloc] = gc;
                sd->owned[nloc] = (i >= i0 + d && i < i1 - d && j >= j0 + d && j < j1 - d && k >= k0 + d && k < k1 - d);
                g2l[gc] = nloc;
                nloc++;
            }
    sd->nloc = nloc;
    int64_t nrow = 4 * (int64_t)nloc;
    sink sk = {0};
    size_t cap2 = 0; term *rows = NULL; int64_t nnz = 0;
    sd->rp = malloc(sizeof(int64_t) * (nrow + 1));
    sd->rp[0] = 0;
    for (int l = 0; l < nloc; l++) {
        int64_t gc = sd->gcell[l];
        int ii = (int)(gc % n), jj = (int)((gc / n) % n), kk = (int)((gc / ((int64_t)n * n)) % g->nr);
        int pp = (int)(gc / ((int64_t)n * n * g->nr));
        for (int c = 0; c < 4; c++) {
            sk.n = 0;
            emit_row(cx, &sk, pp, ii, jj, kk, c);
            size_t m = 0;
            for (size_t a = 0; a < sk.n; a++) {
                int64_t gcol = sk.t[a].col;
                int32_t lc = g2l[gcol / 4];
                if (lc < 0) continue;
                sk.t[m].col = 4 * (int64_t)lc + gcol % 4; sk.t[m].w = sk.t[a].w; m++;
            }
            m = merge_terms(sk.t, m);
            if ((size_t)nnz + m > cap2) {
                cap2 = cap2 ? 2 * cap2 + m : 64 * (size_t)nrow + m;
                rows = realloc(rows, cap2 * sizeof(term));
            }
            memcpy(rows + nnz, sk.t, m * sizeof(term));
            nnz += m;
            sd->rp[4 * l + c + 1] = nnz;
        }
    }
    free(sk.t);
    sd->ci = malloc(sizeof(int32_t) * (nnz + 1));
    sd->v = malloc(sizeof(double) * (nnz + 1));
    sd->diag = malloc(sizeof(int64_t) * (nrow + 1));
    for (int64_t a = 0; a < nnz; a++) { sd->ci[a] = (int32_t)rows[a].col; sd->v[a] = rows[a].w; }
    free(rows);
    for (int l = 0; l < nloc; l++) g2l[sd->gcell[l]] = -1;
    return ilu0(nrow, sd->rp, sd->ci, sd->v, sd->diag);
}

static int onelevel_setup(const ref_grid *g, const ref_op *op, const int sub[3], int overlap, int precision, onelevel **out) {
    seam_tab st; ctx cx;
    *out = NULL;
    if (overlap < 0 || overlap > 1) return REF_EINVAL;
    if (sub[0] < 1 || sub[1] < 1 || sub[2] < 1 || g->n % sub[0] || g->n % sub[1] || g->nr % sub[2]) return REF_EINVAL;
    int rc = make_ctx(g, op, &st, &cx);
    if (rc) return rc;
    onelevel *ol = calloc(1, sizeof(onelevel));
    ol->g = *g; ol->op = *op; ol->overlap = overlap; ol->precision = precision;
    for (int a = 0; a < 3; a++) ol->sub[a] = sub[a];
    ol->nb[0] = g->n / sub[0]; ol->nb[1] = g->n / sub[1]; ol->nb[2] = g->nr / sub[2];
    ol->nsd = 6 * ol->nb[0] * ol->nb[1] * ol->nb[2];
    ol->sd = calloc(ol->nsd, sizeof(subdomain));
    int64_t ncell = 6 * (int64_t)g->n * g->n * g->nr;
    int32_t *g2l = malloc(sizeof(int32_t) * ncell);
    for (int64_t a = 0; a < ncell; a++) g2l[a] = -1;
    for (int s = 0; s < ol->nsd && rc == REF_OK; s++) rc = build_subdomain(&cx, ol, s, g2l);
    free(g2l);
    free_seams(&st);
    if (rc) { ol->nsd = ol->nsd; free_onelevel(ol); return rc; }
    if (precision == 1) /* factors computed in FP64, stored in FP32 */
        for (int s = 0; s < ol->nsd; s++) {
            subdomain *d = &ol->sd[s];
            for (int64_t a = 0; a < d->rp[4 * (int64_t)d->nloc]; a++) d->v[a] = (double)(float)d->v[a];
        }
    *out = ol;
    return REF_OK;
}

/* y = sum_i (R_i^0)^T (L_i U_i)^{-1} R_i^delta x  (eq. onelevel, ILU(0)). */
static void onelevel_apply(const onelevel *ol, const double *x, double *y) {
    int64_t maxrow = 0;
    for (int s = 0; s < ol->nsd; s++) if (4 * (int64_t)ol->sd[s].nloc > maxrow) maxrow = 4 * (int64_t)ol->sd[s].nloc;
    double *t = malloc(sizeof(double) * (maxrow + 1));
    float *tf = malloc(sizeof(float) * (maxrow + 1));
    for (int s = 0; s < ol->nsd; s++) {
        const subdomain *d = &ol->sd[s];
        int64_t nrow = 4 * (int64_t)d->nloc;
        for (int l = 0; l < d->nloc; l++)
            for (int c = 0; c < 4; c++) t[4 * l + c] = x[4 * d->gcell[l] + c];
        if (ol->precision == 0) {
            for (int64_t i = 0; i < nrow; i++) {             /* L z = t, unit diagonal */
                double acc = t[i];
                for (int64_t q = d->rp[i]; q < d->diag[i]; q++) acc -= d->v[q] * t[d->ci[q]];
                t[i] = acc;
            }
            for (int64_t i = nrow - 1; i >= 0; i--) {        /* U y = z */
                double acc = t[i];
                for (int64_t q = d->diag[i] + 1; q < d->rp[i + 1]; q++) acc -= d->v[q] * t[d->ci[q]];
                t[i] = acc / d->v[d->diag[i]];
            }
        } else {  /* FP32 sweeps with FP32 accumulation */
            for (int64_t i = 0; i < nrow; i++) tf[i] = (float)t[i];
            for (int64_t i = 0; i < nrow; i++) {
                float acc = tf[i];
                for (int64_t q = d->rp[i]; q < d->diag[i]; q++) acc -= (float)d->v[q] * tf[d->ci[q]];
                tf[i] = acc;
            }
            for (int64_t i = nrow - 1; i >= 0; i--) {
                float acc = tf[i];
                for (int64_t q = d->diag[i] + 1; q < d->rp[i + 1]; q++) acc -= (float)d->v[q] * tf[d->ci[q]];
                tf[i] = acc / (float)d->v[d->diag[i]];
            }
            for (int64_t i = 0; i < nrow; i++) t[i] = (double)tf[i];
        }
        for (int l = 0; l < d->nloc; l++)
            if (d->owned[l])
                for (int c = 0; c < 4; c++) y[4 * d->gcell[l] + c] = t[4 * l + c];
    }
    free(t); free(tf);
}

/* ----------------------------------------------------------------- solver */
typedef struct {
    int64_t nrow; int64_t *rp; int32_t *ci; double *v;
} csr;

static void csr_free(csr *a) { free(a->rp); free(a->ci); free(a->v); }

static int csr_build(const ref_grid *g, const ref_op *op, csr *a) {
    a->nrow = 24 * (int64_t)g->n * g->n * g->nr;
    a->rp = malloc(sizeof(int64_t) * (a->nrow + 1));
    int rc = ref_assemble(g, op, a->rp, NULL, NULL);
    if (rc) return rc;
    a->ci = malloc(sizeof(int32_t) * a->rp[a->nrow]);
    a->v = malloc(sizeof(double) * a->rp[a->nrow]);
    return ref_assemble(g, op, a->rp, a->ci, a->v);
}

static void csr_mv(const csr *a, const double *x, double *y) {
    for (int64_t i = 0; i < a->nrow; i++) {
        double acc = 0.0;
        for (int64_t q = a->rp[i]; q < a->rp[i + 1]; q++) acc += a->v[q] * x[a->ci[q]];
        y[i] = acc;
    }
}

typedef struct ref_pc ref_pc;
struct ref_pc {
    int levels;                 /* 0 none, 1 one-level, 2 two-level, 3 three-level */
    ref_grid g; ref_op op;
    onelevel *fine;
    csr Af;                     /* fine operator (used in x - A_f w) */
    /* coarse level */
    ref_grid gc; csr Ac; onelevel *coarse; double *vc; /* coarse volumes */
    double coarse_rtol; int coarse_restart, coarse_maxit;
    int precision;
    int64_t inner_iters;        /* total inner iterations since last reset */
    /* levels = 3 (Sec. 3.3: the hybrid construction repeated on the coarser
     * mesh): the coarse solve is preconditioned by this two-level hybrid of
     * the coarse grid instead of the one-level `coarse`, and is flexible */
    ref_pc *inner;
};

typedef struct { int32_t restart, maxit, flexible; double rtol, atol; } ref_gmres_opts;
typedef struct { int32_t iters, restarts; int64_t inner_iters; double relres_true, relres_est; } ref_gmres_stats;

static double nrm2(int64_t n, const double *x) { double s = 0; for (int64_t i = 0; i < n; i++) s += x[i] * x[i]; return sqrt(s); }
static double dotn(int64_t n, const double *x, const double *y) { double s = 0; for (int64_t i = 0; i < n; i++) s += x[i] * y[i]; return s; }

static void pc_apply(ref_pc *pc, const double *x, double *y);

/* Project the pressure component to zero volume-weighted mean (reading R9;
 * the Neumann problem's solvability condition, Sec. 3.1). */
static void project_p(int64_t ncell, const double *vol, double *b) {
    double s = 0, v = 0;
    for (int64_t c = 0; c < ncell; c++) { s += vol[c] * b[4 * c + 3]; v += vol[c]; }
    double m = s / v;
    for (int64_t c = 0; c < ncell; c++) b[4 * c + 3] -= m;
}

/* Right-preconditioned restarted GMRES(m) (or flexible GMRES) with modified
 * Gram-Schmidt and Givens rotations; stops when the residual estimate is at
 * most max(atol, rtol * ||b - A x0||) (Sec. 3.3, the stopping rule after
 * eq. newlinear). */
static int gmres_core(const csr *A, ref_pc *pc, const ref_gmres_opts *o, const double *b, double *x, ref_gmres_stats *stt,
                      double *hist, int hist_len) {
    int64_t n = A->nrow;
    int m = o->restart;
    if (m < 1 || o->maxit < 1) return REF_EINVAL;
    double *V = malloc(sizeof(double) * n * (m + 1));
    double *Z = o->flexible ? malloc(sizeof(double) * n * m) : NULL;
    double *w = malloc(sizeof(double) * n), *z = malloc(sizeof(double) * n), *r = malloc(sizeof(double) * n);
    double *H = calloc((size_t)(m + 1) * m, sizeof(double)), *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *gv = malloc(sizeof(double) * (m + 1)), *yv = malloc(sizeof(double) * m);
    int rc = REF_OK;
    csr_mv(A, x, r);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - r[i];
    double beta0 = nrm2(n, r);
    if (!isfinite(beta0)) { rc = REF_EBREAKDOWN; goto done; }
    double tol = fmax(o->atol, o->rtol * beta0);
    int iters = 0, restarts = 0, conv = beta0 <= tol;
    double est = beta0;
    while (!conv && iters < o->maxit) {
        double beta = nrm2(n, r);
        for (int64_t i = 0; i < n; i++) V[i] = r[i] / beta;
        for (int a = 0; a <= m; a++) gv[a] = 0.0;
        gv[0] = beta;
        int jdone = 0;
        for (int j = 0; j < m && iters < o->maxit; j++) {
            double *vj = V + (int64_t)j * n;
            double *zj = o->flexible ? Z + (int64_t)j * n : z;
            pc_apply(pc, vj, zj);
            csr_mv(A, zj, w);
            double anorm = nrm2(n, w);
            for (int i = 0; i <= j; i++) {
                double h = dotn(n, w, V + (int64_t)i * n);
                H[i * m + j] = h;
                for (int64_t q = 0; q < n; q++) w[q] -= h * V[(int64_t)i * n + q];
            }
            double hn = nrm2(n, w);
            H[(j + 1) * m + j] = hn;
            iters++;
            jdone = j + 1;
            if (!isfinite(hn)) { rc = REF_EBREAKDOWN; goto done; }
            for (int i = 0; i < j; i++) {
                double t1 = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                double t2 = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t1; H[(i + 1) * m + j] = t2;
            }
            double a = H[j * m + j], bb = H[(j + 1) * m + j];
            double den = hypot(a, bb);
            cs[j] = a / den; sn[j] = bb / den;
            H[j * m + j] = den; H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            est = fabs(gv[j + 1]);
            if (hist && iters <= hist_len) hist[iters - 1] = est;   /* residual estimate after each Arnoldi step */
            int happy = hn <= 1e-14 * anorm;
            if (!happy) for (int64_t q = 0; q < n; q++) V[(int64_t)(j + 1) * n + q] = w[q] / hn;
            if (est <= tol || happy) { conv = 1; break; }
        }
        /* y = H^{-1} g (upper triangular) */
        for (int i = jdone - 1; i >= 0; i--) {
            double s = gv[i];
            for (int k = i + 1; k < jdone; k++) s -= H[i * m + k] * yv[k];
            yv[i] = s / H[i * m + i];
        }
        if (o->flexible) {
            for (int i = 0; i < jdone; i++) for (int64_t q = 0; q < n; q++) x[q] += yv[i] * Z[(int64_t)i * n + q];
        } else {
            for (int64_t q = 0; q < n; q++) w[q] = 0.0;
            for (int i = 0; i < jdone; i++) for (int64_t q = 0; q < n; q++) w[q] += yv[i] * V[(int64_t)i * n + q];
            pc_apply(pc, w, z);
            for (int64_t q = 0; q < n; q++) x[q] += z[q];
        }
        csr_mv(A, x, r);
        for (int64_t i = 0; i < n; i++) r[i] = b[i] - r[i];
        if (!conv) restarts++;
    }
    if (stt) {
        stt->iters = iters; stt->restarts = restarts;
        stt->relres_true = beta0 > 0 ? nrm2(n, r) / beta0 : 0.0;
        stt->relres_est = beta0 > 0 ? est / beta0 : 0.0;
    }
    if (!conv) rc = REF_ENOTCONV;
done:
    free(V); free(Z); free(w); free(z); free(r); free(H); free(cs); free(sn); free(gv); free(yv);
    return rc;
}

/* Two-level hybrid preconditioner, y = w + M_one^{-1}(x - A_f w) with
 * w = I_c^f A_c^{-1} I_f^c x (eq. coarsesolve, finesolve; reading R9). */
static void twolevel_apply(ref_pc *pc, const double *x, double *y) {
    const ref_grid *g = &pc->g, *gc = &pc->gc;
    int n = g->n, nc = gc->n;
    int64_t ncc = 6 * (int64_t)nc * nc * gc->nr, nf = 24 * (int64_t)n * n * g->nr;
    double *rc = calloc(4 * ncc, sizeof(double)), *ec = calloc(4 * ncc, sizeof(double));
    for (int p = 0; p < 6; p++)
        for (int K = 0; K < gc->nr; K++)
            for (int J = 0; J < nc; J++)
                for (int I = 0; I < nc; I++)
                    for (int c = 0; c < 4; c++) {
                        double s = 0;
                        for (int dk = 0; dk < 2; dk++) for (int dj = 0; dj < 2; dj++) for (int di = 0; di < 2; di++)
                            s += x[unk(g, p, 2 * I + di, 2 * J + dj, 2 * K + dk, c)];
                        rc[unk(gc, p, I, J, K, c)] = s / 8.0;
                    }
    if (pc->op.kind == 0) project_p(ncc, pc->vc, rc);
    ref_pc cpc = {0};
    cpc.levels = 1; cpc.fine = pc->coarse; cpc.g = *gc; cpc.op = pc->op; cpc.precision = pc->precision;
    /* three levels: FGMRES on the coarse grid with its own two-level hybrid */
    ref_gmres_opts o = {pc->coarse_restart, pc->coarse_maxit, pc->inner != NULL, pc->coarse_rtol, 0.0};
    ref_gmres_stats st = {0};
    gmres_core(&pc->Ac, pc->inner ? pc->inner : &cpc, &o, rc, ec, &st, NULL, 0);
    pc->inner_iters += st.iters;
    double *wv = malloc(sizeof(double) * nf), *t = malloc(sizeof(double) * nf);
    for (int p = 0; p < 6; p++)
        for (int k = 0; k < g->nr; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++)
                    for (int c = 0; c < 4; c++)
                        wv[unk(g, p, i, j, k, c)] = ec[unk(gc, p, i / 2, j / 2, k / 2, c)];
    csr_mv(&pc->Af, wv, t);
    for (int64_t q = 0; q < nf; q++) t[q] = x[q] - t[q];
    onelevel_apply(pc->fine, t, y);
    for (int64_t q = 0; q < nf; q++) y[q] += wv[q];
    free(rc); free(ec); free(wv); free(t);
}

/* ---------------------------------------------- FP32 preconditioner path
 * Reading for the mixed-precision form: every operation inside M^{-1} runs in
 * FP32 (C float, FP32 accumulation): the ILU(0) factors are computed in FP64
 * and rounded to FP32, the sweeps, the restriction and prolongation, the
 * preconditioner-internal A_f w (matrix entries rounded to FP32) and the
 * vector operations of the inner coarse GMRES; the inner GMRES's small
 * Hessenberg least-squares problem stays in FP64.  Input and output of
 * M^{-1} are FP64. */
static void csr_mv_f(const csr *a, const float *x, float *y) {
    for (int64_t i = 0; i < a->nrow; i++) {
        float acc = 0.0f;
        for (int64_t q = a->rp[i]; q < a->rp[i + 1]; q++) acc += (float)a->v[q] * x[a->ci[q]];
        y[i] = acc;
    }
}

static void onelevel_apply_f(const onelevel *ol, const float *x, float *y) {
    int64_t maxrow = 0;
    for (int s = 0; s < ol->nsd; s++) if (4 * (int64_t)ol->sd[s].nloc > maxrow) maxrow = 4 * (int64_t)ol->sd[s].nloc;
    float *t = malloc(sizeof(float) * (maxrow + 1));
    for (int s = 0; s < ol->nsd; s++) {
        const subdomain *d = &ol->sd[s];
        int64_t nrow = 4 * (int64_t)d->nloc;
        for (int l = 0; l < d->nloc; l++)
            for (int c = 0; c < 4; c++) t[4 * l + c] = x[4 * d->gcell[l] + c];
        for (int64_t i = 0; i < nrow; i++) {
            float acc = t[i];
            for (int64_t q = d->rp[i]; q < d->diag[i]; q++) acc -= (float)d->v[q] * t[d->ci[q]];
            t[i] = acc;
        }
        for (int64_t i = nrow - 1; i >= 0; i--) {
            float acc = t[i];
            for (int64_t q = d->diag[i] + 1; q < d->rp[i + 1]; q++) acc -= (float)d->v[q] * t[d->ci[q]];
            t[i] = acc / (float)d->v[d->diag[i]];
        }
        for (int l = 0; l < d->nloc; l++)
            if (d->owned[l])
                for (int c = 0; c < 4; c++) y[4 * d->gcell[l] + c] = t[4 * l + c];
    }
    free(t);
}

static float dotf(int64_t n, const float *x, const float *y) { float s = 0.0f; for (int64_t i = 0; i < n; i++) s += x[i] * y[i]; return s; }

/* GMRES(m) right-preconditioned by the FP32 one-level RAS, FP32 vectors
 * (the coarse solve of the mixed-precision two-level preconditioner). */
static void twolevel_apply_ff(ref_pc *pc, const float *x, float *y);

/* As above; with inner != NULL the preconditioner is that coarse-grid
 * two-level hybrid (FP32 throughout) and the iteration is flexible (the
 * preconditioned directions Z are kept and x += Z y). */
static int gmres_core_f(const csr *A, const onelevel *M, ref_pc *inner, int m, int maxit, double rtol, const float *b,
                        float *x, int *iters_out) {
    int64_t n = A->nrow;
    float *V = malloc(sizeof(float) * n * (m + 1)), *w = malloc(sizeof(float) * n), *z = malloc(sizeof(float) * n);
    float *Z = inner ? malloc(sizeof(float) * n * m) : NULL;
    float *r = malloc(sizeof(float) * n);
    double *H = calloc((size_t)(m + 1) * m, sizeof(double)), *cs = malloc(sizeof(double) * m), *sn = malloc(sizeof(double) * m);
    double *gv = malloc(sizeof(double) * (m + 1)), *yv = malloc(sizeof(double) * m);
    csr_mv_f(A, x, r);
    for (int64_t i = 0; i < n; i++) r[i] = b[i] - r[i];
    double beta0 = sqrt((double)dotf(n, r, r)), tol = rtol * beta0;
    int iters = 0, conv = beta0 <= tol;
    while (!conv && iters < maxit) {
        double beta = sqrt((double)dotf(n, r, r));
        for (int64_t i = 0; i < n; i++) V[i] = (float)(r[i] / beta);
        for (int a = 0; a <= m; a++) gv[a] = 0.0;
        gv[0] = beta;
        int jdone = 0;
        for (int j = 0; j < m && iters < maxit; j++) {
            float *zj = inner ? Z + (int64_t)j * n : z;
            if (inner) twolevel_apply_ff(inner, V + (int64_t)j * n, zj);
            else onelevel_apply_f(M, V + (int64_t)j * n, zj);
            csr_mv_f(A, zj, w);
            double anorm = sqrt((double)dotf(n, w, w));
            for (int i = 0; i <= j; i++) {
                float h = dotf(n, w, V + (int64_t)i * n);
                H[i * m + j] = h;
                for (int64_t q = 0; q < n; q++) w[q] -= h * V[(int64_t)i * n + q];
            }
            double hn = sqrt((double)dotf(n, w, w));
            H[(j + 1) * m + j] = hn;
            iters++;
            jdone = j + 1;
            for (int i = 0; i < j; i++) {
                double t1 = cs[i] * H[i * m + j] + sn[i] * H[(i + 1) * m + j];
                double t2 = -sn[i] * H[i * m + j] + cs[i] * H[(i + 1) * m + j];
                H[i * m + j] = t1; H[(i + 1) * m + j] = t2;
            }
            double a = H[j * m + j], bb = H[(j + 1) * m + j], den = hypot(a, bb);
            cs[j] = a / den; sn[j] = bb / den;
            H[j * m + j] = den; H[(j + 1) * m + j] = 0.0;
            gv[j + 1] = -sn[j] * gv[j];
            gv[j] = cs[j] * gv[j];
            int happy = hn <= 1e-14 * anorm;
            if (!happy) for (int64_t q = 0; q < n; q++) V[(int64_t)(j + 1) * n + q] = (float)(w[q] / hn);
            if (fabs(gv[j + 1]) <= tol || happy) { conv = 1; break; }
        }
        for (int i = jdone - 1; i >= 0; i--) {
            double s2 = gv[i];
            for (int k = i + 1; k < jdone; k++) s2 -= H[i * m + k] * yv[k];
            yv[i] = s2 / H[i * m + i];
        }
        if (inner) {
            for (int i = 0; i < jdone; i++) for (int64_t q = 0; q < n; q++) x[q] += (float)yv[i] * Z[(int64_t)i * n + q];
        } else {
            for (int64_t q = 0; q < n; q++) w[q] = 0.0f;
            for (int i = 0; i < jdone; i++) for (int64_t q = 0; q < n; q++) w[q] += (float)yv[i] * V[(int64_t)i * n + q];
            onelevel_apply_f(M, w, z);
            for (int64_t q = 0; q < n; q++) x[q] += z[q];
        }
        csr_mv_f(A, x, r);
        for (int64_t i = 0; i < n; i++) r[i] = b[i] - r[i];
    }
    *iters_out = iters;
    free(V); free(w); free(z); free(Z); free(r); free(H); free(cs); free(sn); free(gv); free(yv);
    return conv ? REF_OK : REF_ENOTCONV;
}

/* The FP32 two-level hybrid on FP32 vectors (restriction, projection, coarse
 * solve, prolongation, x - A_f w, fine sweeps, y = w + ...). */
static void twolevel_apply_ff(ref_pc *pc, const float *x, float *y) {
    const ref_grid *g = &pc->g, *gc = &pc->gc;
    int n = g->n, nc = gc->n;
    int64_t ncc = 6 * (int64_t)nc * nc * gc->nr, nf = 24 * (int64_t)n * n * g->nr;
    float *rc = calloc(4 * ncc, sizeof(float)), *ec = calloc(4 * ncc, sizeof(float));
    float *wv = malloc(sizeof(float) * nf), *t = malloc(sizeof(float) * nf);
    for (int p = 0; p < 6; p++)
        for (int K = 0; K < gc->nr; K++)
            for (int J = 0; J < nc; J++)
                for (int I = 0; I < nc; I++)
                    for (int c = 0; c < 4; c++) {
                        float s2 = 0.0f;
                        for (int dk = 0; dk < 2; dk++) for (int dj = 0; dj < 2; dj++) for (int di = 0; di < 2; di++)
                            s2 += x[unk(g, p, 2 * I + di, 2 * J + dj, 2 * K + dk, c)];
                        rc[unk(gc, p, I, J, K, c)] = s2 * 0.125f;
                    }
    if (pc->op.kind == 0) {
        float sv = 0.0f, v = 0.0f;
        for (int64_t c = 0; c < ncc; c++) { sv += (float)pc->vc[c] * rc[4 * c + 3]; v += (float)pc->vc[c]; }
        float mean = sv / v;
        for (int64_t c = 0; c < ncc; c++) rc[4 * c + 3] -= mean;
    }
    int it = 0;
    gmres_core_f(&pc->Ac, pc->coarse, pc->inner, pc->coarse_restart, pc->coarse_maxit, pc->coarse_rtol, rc, ec, &it);
    pc->inner_iters += it;
    for (int p = 0; p < 6; p++)
        for (int k = 0; k < g->nr; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++)
                    for (int c = 0; c < 4; c++)
                        wv[unk(g, p, i, j, k, c)] = ec[unk(gc, p, i / 2, j / 2, k / 2, c)];
    csr_mv_f(&pc->Af, wv, t);
    for (int64_t q = 0; q < nf; q++) t[q] = x[q] - t[q];
    onelevel_apply_f(pc->fine, t, y);
    for (int64_t q = 0; q < nf; q++) y[q] += wv[q];
    free(rc); free(ec); free(wv); free(t);
}

static void twolevel_apply_f(ref_pc *pc, const double *xd, double *yd) {
    int64_t nf = 24 * (int64_t)pc->g.n * pc->g.n * pc->g.nr;
    float *x = malloc(sizeof(float) * nf), *y = malloc(sizeof(float) * nf);
    for (int64_t q = 0; q < nf; q++) x[q] = (float)xd[q];
    twolevel_apply_ff(pc, x, y);
    for (int64_t q = 0; q < nf; q++) yd[q] = (double)y[q];
    free(x); free(y);
}

static void pc_apply(ref_pc *pc, const double *x, double *y) {
    int64_t n = 24 * (int64_t)pc->g.n * pc->g.n * pc->g.nr;
    if (pc->levels == 0) { memcpy(y, x, sizeof(double) * n); return; }
    if (pc->levels == 1) { onelevel_apply(pc->fine, x, y); return; }
    if (pc->precision == 1) twolevel_apply_f(pc, x, y);  /* two or three levels */
    else twolevel_apply(pc, x, y);
}

/* ------------------------------------------------- exported: preconditioner */
typedef struct { int32_t sub[3]; int32_t overlap; int32_t levels; double coarse_rtol; int32_t coarse_restart, coarse_maxit; int32_t precision; } ref_ras_opts;
void ref_pc_destroy(ref_pc *pc);

int ref_pc_setup(const ref_grid *g, const ref_op *op, const ref_ras_opts *o, ref_pc **out) {
    *out = NULL;
    if (check_grid(g) || !o || o->levels < 0 || o->levels > 3) return REF_EINVAL;
    ref_pc *pc = calloc(1, sizeof(ref_pc));
    pc->levels = o->levels; pc->g = *g; pc->op = *op; pc->precision = o->precision;
    int rc = REF_OK;
    if (o->levels >= 1) rc = onelevel_setup(g, op, o->sub, o->overlap, o->precision, &pc->fine);
    if (!rc && o->levels >= 2) {
        if (g->n % 2 || g->nr % 2 || o->sub[0] % 2 || o->sub[1] % 2 || o->sub[2] % 2) rc = REF_EINVAL;
        if (!rc) {
            pc->gc = *g; pc->gc.n = g->n / 2; pc->gc.nr = g->nr / 2;
            int subc[3] = {o->sub[0] / 2, o->sub[1] / 2, o->sub[2] / 2};
            rc = csr_build(g, op, &pc->Af);
            if (!rc) rc = csr_build(&pc->gc, op, &pc->Ac);
            if (!rc && o->levels == 2) rc = onelevel_setup(&pc->gc, op, subc, o->overlap, o->precision, &pc->coarse);
            if (!rc && o->levels == 3) {  /* the coarse grid's own two-level hybrid, same subdomain count */
                ref_ras_opts oc = *o;
                oc.levels = 2;
                for (int a = 0; a < 3; a++) oc.sub[a] = subc[a];
                rc = ref_pc_setup(&pc->gc, op, &oc, &pc->inner);
            }
            pc->coarse_rtol = o->coarse_rtol; pc->coarse_restart = o->coarse_restart; pc->coarse_maxit = o->coarse_maxit;
            int64_t ncc = 6 * (int64_t)pc->gc.n * pc->gc.n * pc->gc.nr;
            pc->vc = malloc(sizeof(double) * ncc);
            ref_cell_geometry(&pc->gc, NULL, pc->vc);
        }
    }
    if (rc) {
        ref_pc_destroy(pc);
        return rc;
    }
    *out = pc;
    return REF_OK;
}

void ref_pc_destroy(ref_pc *pc) {
    if (!pc) return;
    ref_pc_destroy(pc->inner);
    free_onelevel(pc->fine); free_onelevel(pc->coarse); csr_free(&pc->Af); csr_free(&pc->Ac); free(pc->vc); free(pc);
}

/* The coarse grid's two-level hybrid of a three-level preconditioner (tests). */
ref_pc *ref_pc_inner(ref_pc *pc) { return pc ? pc->inner : NULL; }
int64_t ref_pc_inner_iters(const ref_pc *pc) { return pc ? pc->inner_iters : 0; }

int ref_pc_apply(ref_pc *pc, const double *x, double *y) { pc_apply(pc, x, y); return REF_OK; }

/* Inspection of a one-level subdomain (tests): sizes, then arrays. */
int ref_pc_subdomain(const ref_pc *pc, int coarse, int s, int64_t *nloc, int64_t *nnz,
                     int64_t *gcell, int32_t *owned, int64_t *rp, int32_t *ci, double *v) {
    const onelevel *ol = coarse ? pc->coarse : pc->fine;
    if (!ol || s < 0 || s >= ol->nsd) return REF_EINVAL;
    const subdomain *d = &ol->sd[s];
    *nloc = d->nloc; *nnz = d->rp[4 * (int64_t)d->nloc];
    if (gcell) for (int l = 0; l < d->nloc; l++) { gcell[l] = d->gcell[l]; owned[l] = d->owned[l]; }
    if (rp) {
        for (int64_t a = 0; a <= 4 * (int64_t)d->nloc; a++) rp[a] = d->rp[a];
        for (int64_t a = 0; a < *nnz; a++) { ci[a] = d->ci[a]; v[a] = d->v[a]; }
    }
    return REF_OK;
}

int ref_pc_count(const ref_pc *pc, int coarse) { const onelevel *ol = coarse ? pc->coarse : pc->fine; return ol ? ol->nsd : 0; }

/* --------------------------------------------------------- exported: solve */
/* As ref_gmres_solve, and hist[k] (k < hist_len) receives the residual
 * estimate |g_{j+1}| after the solve's (k+1)-th Arnoldi step. */
int ref_gmres_solve_hist(const ref_grid *g, const ref_op *op, ref_pc *pc, const ref_gmres_opts *o,
                         const double *b, double *x, ref_gmres_stats *st, double *hist, int hist_len) {
    if (check_grid(g) || !op || !o || !b || !x) return REF_EINVAL;
    csr A;
    int rc = csr_build(g, op, &A);
    if (rc) { csr_free(&A); return rc; }
    int64_t n = A.nrow, ncell = n / 4;
    double *bb = malloc(sizeof(double) * n);
    memcpy(bb, b, sizeof(double) * n);
    double *vol = NULL;
    if (op->kind == 0) { vol = malloc(sizeof(double) * ncell); ref_cell_geometry(g, NULL, vol); project_p(ncell, vol, bb); }
    ref_pc none = {0};
    none.g = *g; none.op = *op;
    ref_pc *use = pc ? pc : &none;
    use->inner_iters = 0;
    for (int64_t i = 0; i < n; i++) if (!isfinite(bb[i]) || !isfinite(x[i])) { rc = REF_EBREAKDOWN; goto out; }
    rc = gmres_core(&A, use, o, bb, x, st, hist, hist_len);
    if (st) st->inner_iters = use->inner_iters;
    if (op->kind == 0 && rc >= 0) project_p(ncell, vol, x); /* remove the null-space component */
out:
    free(bb); free(vol); csr_free(&A);
    return rc;
}

int ref_gmres_solve(const ref_grid *g, const ref_op *op, ref_pc *pc, const ref_gmres_opts *o,
                    const double *b, double *x, ref_gmres_stats *st) {
    return ref_gmres_solve_hist(g, op, pc, o, b, x, st, NULL, 0);
}

/* ILU(0) of an arbitrary CSR matrix with sorted columns (tests). */
int ref_ilu0_csr(int64_t nrow, const int64_t *rp, const int32_t *ci, double *v) {
    int64_t *diag = malloc(sizeof(int64_t) * (size_t)(nrow + 1));
    int rc = ilu0(nrow, rp, ci, v, diag);
    free(diag);
    return rc;
}

/* One subdomain's local solve y_i = (L_i U_i)^{-1} R_i x at full size without
 * building the others (sampled checks): writes the owned cells of y only.
 * precision = 1: factors rounded to FP32 and FP32 sweeps, as in the FP32
 * one-level preconditioner. */
int ref_subdomain_solve_p(const ref_grid *g, const ref_op *op, const int32_t sub[3], int overlap, int s,
                          int precision, const double *x, double *y) {
    seam_tab st; ctx cx;
    if (overlap < 0 || overlap > 1) return REF_EINVAL;
    if (sub[0] < 1 || sub[1] < 1 || sub[2] < 1 || g->n % sub[0] || g->n % sub[1] || g->nr % sub[2]) return REF_EINVAL;
    int rc = make_ctx(g, op, &st, &cx);
    if (rc) return rc;
    onelevel ol = {0};
    ol.g = *g; ol.op = *op; ol.overlap = overlap;
    for (int a = 0; a < 3; a++) ol.sub[a] = sub[a];
    ol.nb[0] = g->n / sub[0]; ol.nb[1] = g->n / sub[1]; ol.nb[2] = g->nr / sub[2];
    ol.nsd = 6 * ol.nb[0] * ol.nb[1] * ol.nb[2];
    if (s < 0 || s >= ol.nsd) { free_seams(&st); return REF_EINVAL; }
    subdomain *all = calloc(ol.nsd, sizeof(subdomain));
    ol.sd = all;
    int64_t ncell = 6 * (int64_t)g->n * g->n * g->nr;
    int32_t *g2l = malloc(sizeof(int32_t) * ncell);
    for (int64_t a = 0; a < ncell; a++) g2l[a] = -1;
    rc = build_subdomain(&cx, &ol, s, g2l);
    free(g2l);
    if (!rc) {
        onelevel one = ol;
        one.sd = &all[s]; one.nsd = 1;
        one.precision = precision == 1;
        if (one.precision) /* factors computed in FP64, stored in FP32, as in onelevel_setup */
            for (int64_t a = 0; a < all[s].rp[4 * (int64_t)all[s].nloc]; a++) all[s].v[a] = (double)(float)all[s].v[a];
        onelevel_apply(&one, x, y);
    }
    subdomain *d = &all[s];
    free(d->gcell); free(d->owned); free(d->rp); free(d->ci); free(d->v); free(d->diag);
    free(all);
    free_seams(&st);
    return rc;
}

int ref_subdomain_solve(const ref_grid *g, const ref_op *op, const int32_t sub[3], int overlap, int s,
                        const double *x, double *y) {
    return ref_subdomain_solve_p(g, op, sub, overlap, s, 0, x, y);
}

/* Step 3 of the time step (Sec. 3.1, eq. ubtilde): from a solution x = (u~, P)
 * return out = (u~ - dt * grad_h P, D_f F) where grad_h P at a cell centre is
 * sum_m g^m (dP/dq^m) with central differences (ghosts across panel edges and
 * walls as in the operator), and D_f F is the finite-volume divergence of the
 * corrected face fluxes F = (flux of u~) - dt (face gradient flux of P), i.e.
 * the pressure row of A x; it vanishes when the P-rows of A x = b hold with
 * b_P = 0 (discrete divergence-free at faces). */
int ref_project(const ref_grid *g, const ref_op *op, const double *x, double *out) {
    seam_tab st; ctx cx;
    if (op && op->kind == 2) return REF_EINVAL;   /* Step 3 belongs to the VP and BP systems */
    int rc = make_ctx(g, op, &st, &cx);
    if (rc) return rc;
    sink s = {0}; s.mode = 1; s.x = x;
    int n = g->n;
    double h = hs_of(g), hr = hr_of(g);
    for (int p = 0; p < 6; p++)
        for (int k = 0; k < g->nr; k++)
            for (int j = 0; j < n; j++)
                for (int i = 0; i < n; i++) {
                    double d[3];
                    s.acc = 0; emit_x(&cx, &s, p, i + 1, j, k, 3, 0.5 / h); emit_x(&cx, &s, p, i - 1, j, k, 3, -0.5 / h); d[0] = s.acc;
                    s.acc = 0; emit_x(&cx, &s, p, i, j + 1, k, 3, 0.5 / h); emit_x(&cx, &s, p, i, j - 1, k, 3, -0.5 / h); d[1] = s.acc;
                    s.acc = 0; emit_x(&cx, &s, p, i, j, k + 1, 3, 0.5 / hr); emit_x(&cx, &s, p, i, j, k - 1, 3, -0.5 / hr); d[2] = s.acc;
                    metric m; metric_at(p, xi_of(g, i), xi_of(g, j), r_of(g, k), &m);
                    for (int c = 0; c < 3; c++) {
                        double gr = d[0] * m.gcon[0][c] + d[1] * m.gcon[1][c] + d[2] * m.gcon[2][c];
                        out[unk(g, p, i, j, k, c)] = x[unk(g, p, i, j, k, c)] - op->dt * gr;
                    }
                    s.acc = 0;
                    emit_row(&cx, &s, p, i, j, k, 3);
                    out[unk(g, p, i, j, k, 3)] = s.acc;
                }
    free_seams(&st);
    return REF_OK;
}
