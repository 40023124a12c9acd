/*
 * oracle.c -- plain fp64 CPU reference for the Icarus finite-volume MHD update.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle that the HIP path is checked
 * against.  Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline
 * leg may load it.  It shares no code with the HIP library.
 *
 * What it computes (paper Sect. 2.1: ideal MHD in the frame co-rotating with
 * the Sun, TVDLF scheme with a Woodward-type limiter, second order in space
 * and time, two ghost layers):
 *   - conserved <-> primitive variables and the fast magnetosonic speed;
 *   - the ideal-MHD flux along one coordinate direction;
 *   - the limited slope of one primitive on a non-uniform coordinate: the
 *     monotonised-central limiter (the Woodward & Colella form, the paper's
 *     choice), minmod or van Leer (the paper names further limiters among the
 *     combinations its code offers);
 *   - the local Lax-Friedrichs (Rusanov) interface flux;
 *   - the spatial operator L(U) of a ghosted patch: flux differences over the
 *     finite volume plus the spherical hoop terms, Coriolis, centrifugal and
 *     solar-gravity sources;
 *   - the Hancock predictor operator: the same differences of each cell's own
 *     physical fluxes at its reconstructed face states (no interface solver);
 *   - the CFL rate, and the per-cell refinement-indicator quantities
 *     (Loehner-type second-derivative estimator and div V);
 *   - the discrete divergence of B per cell (for the parabolic cleaning).
 *
 * Everything is written straight from the equations with no blocking, no
 * fusion and no precomputed reciprocals.  Divisions are divisions.  Build with
 * -O2 -ffp-contract=off (no FMA contraction, IEEE division and sqrt).
 *
 * Layout of a ghosted patch: U[v][k+2][j+2][i+2], v in 0..7, i (r or x)
 * fastest, two ghost layers on every side, sizes (nk+4)(nj+4)(ni+4).  Only the
 * face ghost slabs are read (the scheme is dimension by dimension, so edge and
 * corner ghosts never enter).
 *
 * Variables: U = (rho, m_r, m_theta, m_phi, E, B_r, B_theta, B_phi),
 *            W = (rho, v_r, v_theta, v_phi, p, B_r, B_theta, B_phi),
 * code units with mu_0 = 1, E = p/(gamma-1) + rho v^2/2 + B^2/2.  A patch
 * with nv = 9 carries the CME density tracer as a ninth conserved variable
 * rho s (primitive s, the CME mass fraction): advected with the flow by the
 * same TVDLF flux (rho s v_n and the same c_max), no source term.
 */
#include <math.h>
#include <stddef.h>
#include <string.h>
#include <stdlib.h>

#define NV 8        /* MHD variables */
#define NVMAX 9     /* with the CME density tracer rho s */

typedef struct {
    int ni, nj, nk;        /* interior cells */
    int cartesian;         /* 0: spherical (r, theta, phi); 1: cartesian (x, y, z) */
    const double *f0;      /* faces along direction 0, faces -2..ni+2 stored at [0..ni+4] */
    const double *f1;      /* faces along direction 1 */
    const double *f2;      /* faces along direction 2 */
    double gamma;
    double omega;          /* rotation rate of the frame about the theta = 0 axis */
    double gm;             /* G * M_sun */
    int limiter;           /* 0 monotonised central, 1 minmod, 2 van Leer */
    int nv;                /* 8, or 9 with the density tracer */
} ora_patch;

/* ------------------------------------------------------------------------ */
/* pointwise physics                                                         */
/* ------------------------------------------------------------------------ */

void ora_prim(const double *u, double *w, double gamma)
{
    double rho = u[0];
    double vr = u[1] / rho, vt = u[2] / rho, vp = u[3] / rho;
    double kin = 0.5 * rho * (vr * vr + vt * vt + vp * vp);
    double mag = 0.5 * (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]);
    w[0] = rho;
    w[1] = vr;
    w[2] = vt;
    w[3] = vp;
    w[4] = (gamma - 1.0) * (u[4] - kin - mag);
    w[5] = u[5];
    w[6] = u[6];
    w[7] = u[7];
}

void ora_cons(const double *w, double *u, double gamma)
{
    double rho = w[0];
    double v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    double b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
    u[0] = rho;
    u[1] = rho * w[1];
    u[2] = rho * w[2];
    u[3] = rho * w[3];
    u[4] = w[4] / (gamma - 1.0) + 0.5 * rho * v2 + 0.5 * b2;
    u[5] = w[5];
    u[6] = w[6];
    u[7] = w[7];
}

/* fast magnetosonic speed along direction d:
 * c_f^2 = 1/2 [ (g p + B^2)/rho + sqrt( ((g p + B^2)/rho)^2 - 4 g p B_d^2 / rho^2 ) ] */
double ora_fast_speed(const double *w, int d, double gamma)
{
    double rho = w[0], p = w[4];
    double b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
    double bd = w[5 + d];
    double a = (gamma * p + b2) / rho;
    double disc = a * a - 4.0 * gamma * p * bd * bd / (rho * rho);
    if (disc < 0.0) disc = 0.0;
    return sqrt(0.5 * (a + sqrt(disc)));
}

/* ideal-MHD flux along direction d (normal index n = d) */
void ora_flux(const double *w, int d, double gamma, double *f)
{
    double rho = w[0], p = w[4];
    const double *v = w + 1;
    const double *b = w + 5;
    double v2 = v[0] * v[0] + v[1] * v[1] + v[2] * v[2];
    double b2 = b[0] * b[0] + b[1] * b[1] + b[2] * b[2];
    double ptot = p + 0.5 * b2;
    double E = p / (gamma - 1.0) + 0.5 * rho * v2 + 0.5 * b2;
    double vn = v[d], bn = b[d];
    double vb = v[0] * b[0] + v[1] * b[1] + v[2] * b[2];
    f[0] = rho * vn;
    for (int c = 0; c < 3; ++c) {
        f[1 + c] = rho * vn * v[c] - bn * b[c] + (c == d ? ptot : 0.0);
        f[5 + c] = vn * b[c] - bn * v[c];
    }
    f[5 + d] = 0.0;
    f[4] = (E + ptot) * vn - bn * vb;
}

/* Rusanov (local Lax-Friedrichs) interface flux */
void ora_rusanov(const double *wl, const double *wr, int d, double gamma, double *f)
{
    double fl[NV], fr[NV], ul[NV], ur[NV];
    ora_flux(wl, d, gamma, fl);
    ora_flux(wr, d, gamma, fr);
    ora_cons(wl, ul, gamma);
    ora_cons(wr, ur, gamma);
    double cl = fabs(wl[1 + d]) + ora_fast_speed(wl, d, gamma);
    double cr = fabs(wr[1 + d]) + ora_fast_speed(wr, d, gamma);
    double c = cl > cr ? cl : cr;
    for (int v = 0; v < NV; ++v)
        f[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * c * (ur[v] - ul[v]);
}

/* the same with the density tracer when nv = 9: s = (rho s) / rho, its flux
 * rho s v_n, and in the interface flux the same c_max as the MHD variables */
static void prim_nv(int nv, const double *u, double *w, double gamma)
{
    ora_prim(u, w, gamma);
    if (nv > NV) w[8] = u[8] / u[0];
}

static void cons_nv(int nv, const double *w, double *u, double gamma)
{
    ora_cons(w, u, gamma);
    if (nv > NV) u[8] = w[0] * w[8];
}

static void flux_nv(int nv, const double *w, int d, double gamma, double *f)
{
    ora_flux(w, d, gamma, f);
    if (nv > NV) f[8] = w[0] * w[8] * w[1 + d];
}

static void rusanov_nv(int nv, const double *wl, const double *wr, int d, double gamma, double *f)
{
    double fl[NVMAX], fr[NVMAX], ul[NVMAX], ur[NVMAX];
    flux_nv(nv, wl, d, gamma, fl);
    flux_nv(nv, wr, d, gamma, fr);
    cons_nv(nv, wl, ul, gamma);
    cons_nv(nv, wr, ur, gamma);
    double cl = fabs(wl[1 + d]) + ora_fast_speed(wl, d, gamma);
    double cr = fabs(wr[1 + d]) + ora_fast_speed(wr, d, gamma);
    double c = cl > cr ? cl : cr;
    for (int v = 0; v < nv; ++v)
        f[v] = 0.5 * (fl[v] + fr[v]) - 0.5 * c * (ur[v] - ul[v]);
}

/* monotonised-central slope on a non-uniform coordinate */
double ora_mc_slope(double wm, double w0, double wp, double xm, double x0, double xp)
{
    double dm = (w0 - wm) / (x0 - xm);
    double dp = (wp - w0) / (xp - x0);
    double dc = (wp - wm) / (xp - xm);
    if (dm * dp <= 0.0) return 0.0;
    double a = fabs(dc);
    if (2.0 * fabs(dm) < a) a = 2.0 * fabs(dm);
    if (2.0 * fabs(dp) < a) a = 2.0 * fabs(dp);
    return dc > 0.0 ? a : -a;
}

/* limited slope by limiter kind (0 monotonised central, 1 minmod, 2 van
 * Leer): with the one-sided differences dm, dp of the primitive, zero where
 * they differ in sign or one vanishes; otherwise
 *   minmod:   the one of smaller magnitude,
 *   van Leer: their harmonic mean 2 dm dp / (dm + dp). */
double ora_slope(int limiter, double wm, double w0, double wp, double xm, double x0, double xp)
{
    if (limiter == 0) return ora_mc_slope(wm, w0, wp, xm, x0, xp);
    double dm = (w0 - wm) / (x0 - xm);
    double dp = (wp - w0) / (xp - x0);
    if (dm * dp <= 0.0) return 0.0;
    if (limiter == 1) return fabs(dm) < fabs(dp) ? dm : dp;
    return 2.0 * dm * dp / (dm + dp);
}

/*
 * Source terms of a cell with primitive state w (spherical geometry only).
 *   rtinv = 1/r in its finite-volume form 3(r+^2 - r-^2) / (2(r+^3 - r-^3))
 *   ctil  = cot(theta) in its finite-volume form (sin t+ - sin t-)/(cos t- - cos t+)
 *   rc, sc, cc = centre radius, sin and cos of the centre colatitude
 * Hoop terms: the parts of the divergence of the momentum tensor
 * rho v v - B B + p_tot I and of the induction tensor v B - B v that are not
 * flux differences in spherical components.  Frame: Coriolis -2 Omega x v and
 * centrifugal -Omega x (Omega x r) with Omega along theta = 0; gravity
 * -GM/r^2 along r; their work in the energy equation (Coriolis does none).
 */
void ora_sources(const double *w, double rtinv, double ctil, double rc, double sc, double cc,
                 double omega, double gm, double *S)
{
    double rho = w[0], vr = w[1], vt = w[2], vp = w[3], pr = w[4];
    double br = w[5], bt = w[6], bp = w[7];
    double ptot = pr + 0.5 * (br * br + bt * bt + bp * bp);
    double g = -gm / (rc * rc);
    double Om = omega;
    for (int v = 0; v < NV; ++v) S[v] = 0.0;
    S[1] = rtinv * (rho * (vt * vt + vp * vp) - (bt * bt + bp * bp) + 2.0 * ptot);
    S[2] = rtinv * (-(rho * vr * vt - br * bt) + ctil * (rho * vp * vp - bp * bp + ptot));
    S[3] = -rtinv * ((rho * vp * vr - bp * br) + ctil * (rho * vp * vt - bp * bt));
    S[6] = rtinv * (vr * bt - vt * br);
    S[7] = -rtinv * ((vp * br - bp * vr) + ctil * (vp * bt - bp * vt));
    S[1] += rho * (2.0 * Om * sc * vp + Om * Om * rc * sc * sc) + rho * g;
    S[2] += rho * (2.0 * Om * cc * vp + Om * Om * rc * sc * cc);
    S[3] += -2.0 * Om * rho * (sc * vr + cc * vt);
    S[4] += rho * vr * g + rho * Om * Om * rc * sc * (vr * sc + vt * cc);
}

/* ------------------------------------------------------------------------ */
/* patch helpers                                                             */
/* ------------------------------------------------------------------------ */

static size_t gix(const ora_patch *p, int v, int i, int j, int k)
{
    size_t ni4 = (size_t)p->ni + 4, nj4 = (size_t)p->nj + 4, nk4 = (size_t)p->nk + 4;
    return (((size_t)v * nk4 + (size_t)(k + 2)) * nj4 + (size_t)(j + 2)) * ni4 + (size_t)(i + 2);
}

static const double *faces(const ora_patch *p, int d)
{
    return d == 0 ? p->f0 : (d == 1 ? p->f1 : p->f2);
}

/* face m of direction d (m = -2..n+2) */
static double face(const ora_patch *p, int d, int m) { return faces(p, d)[m + 2]; }
/* centre of cell m (arithmetic midpoint of its faces) */
static double centre(const ora_patch *p, int d, int m)
{
    return 0.5 * (face(p, d, m) + face(p, d, m + 1));
}

static void cell_prim(const ora_patch *p, const double *U, int i, int j, int k, double *w)
{
    double u[NVMAX];
    for (int v = 0; v < p->nv; ++v) u[v] = U[gix(p, v, i, j, k)];
    prim_nv(p->nv, u, w, p->gamma);
}

/* Reconstruct cell c (index along d; the other two indices fixed) at its two
 * faces.  Slopes per primitive by the MC limiter; if any reconstructed
 * density or pressure is not positive, the cell falls back to zero slope in
 * this direction for all variables. */
static void reconstruct(const ora_patch *p, const double *U, int d, int c, int a, int b,
                        double *w_lo, double *w_hi)
{
    int idx[3];
    double wm[NVMAX], w0[NVMAX], wp[NVMAX];
    idx[(d + 1) % 3] = a;
    idx[(d + 2) % 3] = b;
    idx[d] = c - 1; cell_prim(p, U, idx[0], idx[1], idx[2], wm);
    idx[d] = c;     cell_prim(p, U, idx[0], idx[1], idx[2], w0);
    idx[d] = c + 1; cell_prim(p, U, idx[0], idx[1], idx[2], wp);
    double xm = centre(p, d, c - 1), x0 = centre(p, d, c), xp = centre(p, d, c + 1);
    double flo = face(p, d, c), fhi = face(p, d, c + 1);
    double s[NVMAX];
    for (int v = 0; v < p->nv; ++v) {
        s[v] = ora_slope(p->limiter, wm[v], w0[v], wp[v], xm, x0, xp);
        w_lo[v] = w0[v] - s[v] * (x0 - flo);
        w_hi[v] = w0[v] + s[v] * (fhi - x0);
    }
    if (w_lo[0] <= 0.0 || w_hi[0] <= 0.0 || w_lo[4] <= 0.0 || w_hi[4] <= 0.0) {
        for (int v = 0; v < p->nv; ++v) { w_lo[v] = w0[v]; w_hi[v] = w0[v]; }
    }
}

/* geometric factors A_face / V of cell (i, j, k) in direction d at its lower
 * (am) and upper (ap) face.  Spherical cell [r-,r+]x[t-,t+]x[p-,p+]:
 *   V   = (r+^3 - r-^3)/3 (cos t- - cos t+) dphi
 *   A_r = r_f^2 (cos t- - cos t+) dphi
 *   A_t = (r+^2 - r-^2)/2 sin t_f dphi
 *   A_p = (r+^2 - r-^2)/2 dtheta
 * The ratios are written in the form where the common angular factors have
 * cancelled algebraically.  Cartesian: A/V = 1/dx_d. */
static void metric(const ora_patch *p, int d, int i, int j, int k, double *am, double *ap)
{
    if (p->cartesian) {
        int m = d == 0 ? i : (d == 1 ? j : k);
        *am = *ap = 1.0 / (face(p, d, m + 1) - face(p, d, m));
        return;
    }
    double rm = face(p, 0, i), rp = face(p, 0, i + 1);
    double tm = face(p, 1, j), tp = face(p, 1, j + 1);
    double dr3 = rp * rp * rp - rm * rm * rm;
    double rtinv = 1.5 * (rp * rp - rm * rm) / dr3;   /* (A_r+ - A_r-)/(2V) */
    double dmu = cos(tm) - cos(tp);
    if (d == 0) {
        *am = 3.0 * rm * rm / dr3;
        *ap = 3.0 * rp * rp / dr3;
    } else if (d == 1) {
        *am = rtinv * sin(tm) / dmu;
        *ap = rtinv * sin(tp) / dmu;
    } else {
        double dphi = face(p, 2, k + 1) - face(p, 2, k);
        *am = *ap = rtinv * (tp - tm) / (dmu * dphi);
    }
}

/* ------------------------------------------------------------------------ */
/* the spatial operator                                                      */
/* ------------------------------------------------------------------------ */

/*
 * L(U) on the interior of a ghosted patch.
 *   U   ghosted input, layout above
 *   L   interior output [v][k][j][i]
 *   F0  face fluxes along d=0, [v][k][j][i_face], i_face = 0..ni (face i_face is
 *       the lower face of cell i_face); F1: [v][k][j_face][i]; F2: [v][k_face][j][i].
 *       Any of F0/F1/F2 may be NULL (a temporary buffer is used then).
 * Returns the number of interior cells with rho <= 0, p <= 0 or a non-finite value
 * (-1 if a temporary buffer cannot be allocated).
 */
int ora_rhs(const ora_patch *p, const double *U, double *L, double *F0, double *F1, double *F2)
{
    const int ni = p->ni, nj = p->nj, nk = p->nk;
    const double gamma = p->gamma;
    int bad = 0;
    /* the divergence below reads the face fluxes: a direction whose buffer
     * the caller leaves out gets a temporary one */
    double *own[3] = {NULL, NULL, NULL};
    double **Fs[3] = {&F0, &F1, &F2};
    for (int d = 0; d < 3; ++d)
        if (!*Fs[d]) {
            size_t n = (size_t)p->nv * (nk + (d == 2)) * (nj + (d == 1)) * (ni + (d == 0));
            own[d] = (double *)malloc(n * sizeof(double));
            if (!own[d]) {
                for (int e = 0; e < d; ++e) free(own[e]);
                return -1;
            }
            *Fs[d] = own[d];
        }

    /* interface fluxes, per direction, stored [v][k][j][i] with the face
     * direction extended by one */
    for (int d = 0; d < 3; ++d) {
        double *F = d == 0 ? F0 : (d == 1 ? F1 : F2);
        int fn[3] = {ni, nj, nk};
        fn[d] += 1;
        #pragma omp parallel for schedule(static)
        for (int k = 0; k < fn[2]; ++k) {
            for (int j = 0; j < fn[1]; ++j) {
                for (int i = 0; i < fn[0]; ++i) {
                    int c[3] = {i, j, k};
                    int a = c[(d + 1) % 3], b = c[(d + 2) % 3];
                    double lo_m[NVMAX], hi_m[NVMAX], lo_p[NVMAX], hi_p[NVMAX], f[NVMAX];
                    /* face c[d] lies between cells c[d]-1 (left) and c[d] (right) */
                    reconstruct(p, U, d, c[d] - 1, a, b, lo_m, hi_m);
                    reconstruct(p, U, d, c[d], a, b, lo_p, hi_p);
                    rusanov_nv(p->nv, hi_m, lo_p, d, gamma, f);
                    for (int v = 0; v < p->nv; ++v)
                        F[(((size_t)v * fn[2] + k) * fn[1] + j) * fn[0] + i] = f[v];
                }
            }
        }
    }

    /* divergence + sources per interior cell */
    #pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int k = 0; k < nk; ++k) {
        for (int j = 0; j < nj; ++j) {
            for (int i = 0; i < ni; ++i) {
                double w[NVMAX];
                cell_prim(p, U, i, j, k, w);
                int ok = w[0] > 0.0 && w[4] > 0.0;
                for (int v = 0; v < p->nv; ++v) ok = ok && isfinite(w[v]);
                if (!ok) bad += 1;

                double acc[NVMAX];
                for (int v = 0; v < p->nv; ++v) acc[v] = 0.0;
                for (int d = 0; d < 3; ++d) {
                    double *F = d == 0 ? F0 : (d == 1 ? F1 : F2);
                    int fn[3] = {ni, nj, nk};
                    fn[d] += 1;
                    int cl[3] = {i, j, k}, cu[3] = {i, j, k};
                    cu[d] += 1;
                    double am, ap;
                    metric(p, d, i, j, k, &am, &ap);
                    for (int v = 0; v < p->nv; ++v) {
                        double fl = F[(((size_t)v * fn[2] + cl[2]) * fn[1] + cl[1]) * fn[0] + cl[0]];
                        double fu = F[(((size_t)v * fn[2] + cu[2]) * fn[1] + cu[1]) * fn[0] + cu[0]];
                        acc[v] -= ap * fu - am * fl;
                    }
                }

                if (!p->cartesian) {
                    double rm = face(p, 0, i), rp = face(p, 0, i + 1);
                    double tm = face(p, 1, j), tp = face(p, 1, j + 1);
                    double rtinv = 1.5 * (rp * rp - rm * rm) / (rp * rp * rp - rm * rm * rm);
                    double dmu = cos(tm) - cos(tp);
                    double ctil = (sin(tp) - sin(tm)) / dmu;
                    double tc = centre(p, 1, j);
                    double S[NV];
                    ora_sources(w, rtinv, ctil, centre(p, 0, i), sin(tc), cos(tc), p->omega, p->gm, S);
                    for (int v = 0; v < NV; ++v) acc[v] += S[v];      /* no source of rho s */
                }
                for (int v = 0; v < p->nv; ++v)
                    L[(((size_t)v * nk + k) * nj + j) * ni + i] = acc[v];
            }
        }
    }
    for (int d = 0; d < 3; ++d) free(own[d]);
    return bad;
}

/*
 * Hancock predictor operator on the interior of a ghosted patch: for each
 * cell and direction, the cell's reconstructed face states (limiter as in
 * ora_rhs) give the physical fluxes F(w_lo), F(w_hi) at its own lower and
 * upper faces; L = -(1/V) sum_d [A+ F(w_hi) - A- F(w_lo)] + sources at the
 * cell state.  No interface solver: the predictor U* = U + (dt/2) L gives
 * the half-step state from which the corrector computes the TVDLF fluxes.
 * Returns the number of interior cells with rho <= 0, p <= 0 or a
 * non-finite value.
 */
int ora_rhs_hancock(const ora_patch *p, const double *U, double *L)
{
    const int ni = p->ni, nj = p->nj, nk = p->nk;
    int bad = 0;
    #pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int k = 0; k < nk; ++k) {
        for (int j = 0; j < nj; ++j) {
            for (int i = 0; i < ni; ++i) {
                double w[NVMAX], acc[NVMAX];
                cell_prim(p, U, i, j, k, w);
                int ok = w[0] > 0.0 && w[4] > 0.0;
                for (int v = 0; v < p->nv; ++v) ok = ok && isfinite(w[v]);
                if (!ok) bad += 1;
                for (int v = 0; v < p->nv; ++v) acc[v] = 0.0;
                int c[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    double lo[NVMAX], hi[NVMAX], flo[NVMAX], fhi[NVMAX], am, ap;
                    reconstruct(p, U, d, c[d], c[(d + 1) % 3], c[(d + 2) % 3], lo, hi);
                    flux_nv(p->nv, lo, d, p->gamma, flo);
                    flux_nv(p->nv, hi, d, p->gamma, fhi);
                    metric(p, d, i, j, k, &am, &ap);
                    for (int v = 0; v < p->nv; ++v) acc[v] -= ap * fhi[v] - am * flo[v];
                }
                if (!p->cartesian) {
                    double rm = face(p, 0, i), rp = face(p, 0, i + 1);
                    double tm = face(p, 1, j), tp = face(p, 1, j + 1);
                    double rtinv = 1.5 * (rp * rp - rm * rm) / (rp * rp * rp - rm * rm * rm);
                    double dmu = cos(tm) - cos(tp);
                    double ctil = (sin(tp) - sin(tm)) / dmu;
                    double tc = centre(p, 1, j);
                    double S[NV];
                    ora_sources(w, rtinv, ctil, centre(p, 0, i), sin(tc), cos(tc), p->omega, p->gm, S);
                    for (int v = 0; v < NV; ++v) acc[v] += S[v];
                }
                for (int v = 0; v < p->nv; ++v) L[(((size_t)v * nk + k) * nj + j) * ni + i] = acc[v];
            }
        }
    }
    return bad;
}

/* max over interior cells of sum_d (|v_d| + c_f,d) / dx_d; dx_r = dr,
 * dx_theta = r_c dtheta, dx_phi = r_c sin(theta_c) dphi (spherical). */
double ora_max_rate(const ora_patch *p, const double *U)
{
    double best = 0.0;
    for (int k = 0; k < p->nk; ++k)
        for (int j = 0; j < p->nj; ++j)
            for (int i = 0; i < p->ni; ++i) {
                double w[NVMAX];
                cell_prim(p, U, i, j, k, w);
                double dx[3];
                int m[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) dx[d] = face(p, d, m[d] + 1) - face(p, d, m[d]);
                if (!p->cartesian) {
                    double rc = centre(p, 0, i), tc = centre(p, 1, j);
                    dx[1] = rc * dx[1];
                    dx[2] = rc * sin(tc) * dx[2];
                }
                double rate = 0.0;
                for (int d = 0; d < 3; ++d)
                    rate += (fabs(w[1 + d]) + ora_fast_speed(w, d, p->gamma)) / dx[d];
                if (rate > best) best = rate;
            }
    return best;
}

/*
 * Per-cell refinement-indicator quantities on the interior.
 *   E_rho, E_v : Loehner-type estimator of rho and |v| (per-direction form):
 *       num = sum_d (u+ - 2u + u-)^2
 *       den = sum_d (|u+ - u| + |u - u-| + eps (|u+| + 2|u| + |u-|))^2
 *       E = sqrt(num/den), 0 where den = 0
 *   divv       : (1/V) sum_d (A+ v~+ - A- v~-), v~ the mean of the face-normal
 *                velocities of the two cells sharing the face
 *   divscale   : sum_d (|A+ v~+| + |A- v~-|)/V, the magnitude the sign test is
 *                made against (used to detect near-ties)
 * Outputs are interior arrays [k][j][i].
 */
void ora_indicator(const ora_patch *p, const double *U, double eps,
                   double *E_rho, double *E_v, double *divv, double *divscale)
{
    for (int k = 0; k < p->nk; ++k)
        for (int j = 0; j < p->nj; ++j)
            for (int i = 0; i < p->ni; ++i) {
                double num_r = 0, den_r = 0, num_v = 0, den_v = 0, dv = 0, ds = 0;
                double w0[NVMAX];
                cell_prim(p, U, i, j, k, w0);
                double r0 = w0[0];
                double s0 = sqrt(w0[1] * w0[1] + w0[2] * w0[2] + w0[3] * w0[3]);
                for (int d = 0; d < 3; ++d) {
                    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
                    lo[d] -= 1;
                    hi[d] += 1;
                    double wl[NVMAX], wh[NVMAX];
                    cell_prim(p, U, lo[0], lo[1], lo[2], wl);
                    cell_prim(p, U, hi[0], hi[1], hi[2], wh);
                    double rl = wl[0], rh = wh[0];
                    double sl = sqrt(wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3]);
                    double sh = sqrt(wh[1] * wh[1] + wh[2] * wh[2] + wh[3] * wh[3]);
                    double t;
                    t = rh - 2.0 * r0 + rl;
                    num_r += t * t;
                    t = fabs(rh - r0) + fabs(r0 - rl) + eps * (fabs(rh) + 2.0 * fabs(r0) + fabs(rl));
                    den_r += t * t;
                    t = sh - 2.0 * s0 + sl;
                    num_v += t * t;
                    t = fabs(sh - s0) + fabs(s0 - sl) + eps * (fabs(sh) + 2.0 * fabs(s0) + fabs(sl));
                    den_v += t * t;

                    double vl = 0.5 * (wl[1 + d] + w0[1 + d]);
                    double vh = 0.5 * (w0[1 + d] + wh[1 + d]);
                    double am, ap;
                    metric(p, d, i, j, k, &am, &ap);
                    dv += ap * vh - am * vl;
                    ds += fabs(ap * vh) + fabs(am * vl);
                }
                size_t o = ((size_t)k * p->nj + j) * p->ni + i;
                E_rho[o] = den_r > 0.0 ? sqrt(num_r / den_r) : 0.0;
                E_v[o] = den_v > 0.0 ? sqrt(num_v / den_v) : 0.0;
                divv[o] = dv;
                divscale[o] = ds;
            }
}

/*
 * Discrete div B of every interior cell: (1/V) sum_d [A+ Bt+ - A- Bt-], Bt the
 * mean of the two cells' face-normal field components at the face (the same
 * face-mean form as div V of the indicator).  D is [k][j][i].
 */
void ora_divb(const ora_patch *p, const double *U, double *D)
{
    for (int k = 0; k < p->nk; ++k)
        for (int j = 0; j < p->nj; ++j)
            for (int i = 0; i < p->ni; ++i) {
                double dv = 0.0;
                for (int d = 0; d < 3; ++d) {
                    int lo[3] = {i, j, k}, hi[3] = {i, j, k};
                    lo[d] -= 1;
                    hi[d] += 1;
                    double b0 = U[gix(p, 5 + d, i, j, k)];
                    double bl = 0.5 * (U[gix(p, 5 + d, lo[0], lo[1], lo[2])] + b0);
                    double bh = 0.5 * (b0 + U[gix(p, 5 + d, hi[0], hi[1], hi[2])]);
                    double am, ap;
                    metric(p, d, i, j, k, &am, &ap);
                    dv += ap * bh - am * bl;
                }
                D[((size_t)k * p->nj + j) * p->ni + i] = dv;
            }
}
