// physics.h -- pointwise ideal-MHD physics for the kernels (fp64).
//
// Variables: conserved u = (rho, m0, m1, m2, E, B0, B1, B2), primitive
// w = (rho, v0, v1, v2, p, B0, B1, B2), mu0 = 1, E = p/(g-1) + rho v^2/2 + B^2/2.
// NV = 9 adds the CME density tracer: conserved rho s, primitive s (the CME
// mass fraction), advected with the flow by the same flux (no source).
// Direction 0/1/2 = r/theta/phi (x/y/z in the cartesian test geometry).
#pragma once
#include <hip/hip_runtime.h>

#define DEV __device__ __forceinline__

// Reciprocal of a > 0 (normal): the hardware estimate refined by two
// Newton-Raphson steps x <- x + x (1 - a x); at most one ulp from 1/a.
DEV double rcp_pos(double a)
{
    double x = __builtin_amdgcn_rcp(a);
    double e = fma(-a, x, 1.0);
    x = fma(x, e, x);
    e = fma(-a, x, 1.0);
    return fma(x, e, x);
}

// Square root of x >= 0 (normal or zero): the hardware reciprocal-square-root
// estimate y, then one coupled Goldschmidt iteration on g = x y, h = y / 2 and
// a final Newton correction of g; at most one ulp from sqrt(x).
DEV double sqrt_pos(double x)
{
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y, h = 0.5 * y;
    const double r = fma(-g, h, 0.5);
    g = fma(g, r, g);
    h = fma(h, r, h);
    const double d = fma(-g, g, x);
    g = fma(d, h, g);
    return x > 0.0 ? g : 0.0;
}

// Reciprocals and square roots of the finite-volume update use rcp_pos /
// sqrt_pos (<= 1 ulp); IC_EXACT_MATH selects the IEEE-rounded operations.
#ifdef IC_EXACT_MATH
#define IC_RCP(x) (1.0 / (x))
#define IC_SQRT(x) sqrt(x)
#else
#define IC_RCP(x) rcp_pos(x)
#define IC_SQRT(x) sqrt_pos(x)
#endif

struct Gas {
    double g;       // adiabatic index
    double gm1;     // g - 1
    double igm1;    // 1 / (g - 1)
};

// EXACT: IEEE division (the refinement indicator and the network features,
// whose threshold decisions are kept on the correctly rounded quotient).  The
// tracer fraction s = (rho s) / rho is always the correctly rounded quotient,
// so that s = 1 where rho s = rho.
template <bool EXACT = false, int NV = 8>
DEV void cons_to_prim(const double *u, double *w, const Gas &gs)
{
    const double ir = EXACT ? 1.0 / u[0] : IC_RCP(u[0]);
    w[0] = u[0];
    w[1] = u[1] * ir;
    w[2] = u[2] * ir;
    w[3] = u[3] * ir;
    const double kin = 0.5 * (u[1] * w[1] + u[2] * w[2] + u[3] * w[3]);
    const double mag = 0.5 * (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]);
    w[4] = gs.gm1 * (u[4] - kin - mag);
    w[5] = u[5];
    w[6] = u[6];
    w[7] = u[7];
    if constexpr (NV > 8) w[8] = u[8] / u[0];
}

template <int NV = 8>
DEV void prim_to_cons(const double *w, double *u, const Gas &gs)
{
    const double v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    const double b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
    u[0] = w[0];
    u[1] = w[0] * w[1];
    u[2] = w[0] * w[2];
    u[3] = w[0] * w[3];
    u[4] = w[4] * gs.igm1 + 0.5 * w[0] * v2 + 0.5 * b2;
    u[5] = w[5];
    u[6] = w[6];
    u[7] = w[7];
    if constexpr (NV > 8) u[8] = w[0] * w[8];
}

// Fast magnetosonic speed along direction D.
template <int D>
DEV double fast_speed(const double w[8], const Gas &gs)
{
    const double ir = IC_RCP(w[0]);
    const double b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
    const double gp = gs.g * w[4];
    const double a = (gp + b2) * ir;
    const double bn = w[5 + D];
    double disc = a * a - 4.0 * gp * bn * bn * ir * ir;
    disc = disc > 0.0 ? disc : 0.0;
    return IC_SQRT(0.5 * (a + IC_SQRT(disc)));
}

template <int NV = 8>
DEV bool unphysical(const double *w)
{
    // rho <= 0, p <= 0 or NaN (comparisons with NaN are false)
    bool ok = (w[0] > 0.0) && (w[4] > 0.0);
#pragma unroll
    for (int v = 0; v < NV; ++v) ok = ok && (fabs(w[v]) <= 1.7976931348623157e308);
    return !ok;
}

// Local Lax-Friedrichs (Rusanov) flux along D between left state wl and right
// state wr; with the tracer, its flux rho v_n s takes the same maximum speed.
template <int D, int NV = 8>
DEV void rusanov(const double *wl, const double *wr, double *f, const Gas &gs)
{
    const double vl2 = wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3];
    const double vr2 = wr[1] * wr[1] + wr[2] * wr[2] + wr[3] * wr[3];
    const double bl2 = wl[5] * wl[5] + wl[6] * wl[6] + wl[7] * wl[7];
    const double br2 = wr[5] * wr[5] + wr[6] * wr[6] + wr[7] * wr[7];
    const double ptl = wl[4] + 0.5 * bl2;
    const double ptr = wr[4] + 0.5 * br2;
    const double El = wl[4] * gs.igm1 + 0.5 * wl[0] * vl2 + 0.5 * bl2;
    const double Er = wr[4] * gs.igm1 + 0.5 * wr[0] * vr2 + 0.5 * br2;
    const double vnl = wl[1 + D], vnr = wr[1 + D];
    const double bnl = wl[5 + D], bnr = wr[5 + D];
    const double vbl = wl[1] * wl[5] + wl[2] * wl[6] + wl[3] * wl[7];
    const double vbr = wr[1] * wr[5] + wr[2] * wr[6] + wr[3] * wr[7];
    // fast speeds
    const double irl = IC_RCP(wl[0]), irr = IC_RCP(wr[0]);
    const double gpl = gs.g * wl[4], gpr = gs.g * wr[4];
    const double al = (gpl + bl2) * irl, ar = (gpr + br2) * irr;
    double dl = al * al - 4.0 * gpl * bnl * bnl * irl * irl;
    double dr = ar * ar - 4.0 * gpr * bnr * bnr * irr * irr;
    dl = dl > 0.0 ? dl : 0.0;
    dr = dr > 0.0 ? dr : 0.0;
    const double cfl = IC_SQRT(0.5 * (al + IC_SQRT(dl)));
    const double cfr = IC_SQRT(0.5 * (ar + IC_SQRT(dr)));
    const double sl = fabs(vnl) + cfl, sr = fabs(vnr) + cfr;
    const double c = sl > sr ? sl : sr;
    const double hc = 0.5 * c;

    const double ml = wl[0] * vnl, mr = wr[0] * vnr;
    f[0] = 0.5 * (ml + mr) - hc * (wr[0] - wl[0]);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double fl = ml * wl[1 + q] - bnl * wl[5 + q];
        double fr = mr * wr[1 + q] - bnr * wr[5 + q];
        if (q == D) {
            fl += ptl;
            fr += ptr;
        }
        f[1 + q] = 0.5 * (fl + fr) - hc * (wr[0] * wr[1 + q] - wl[0] * wl[1 + q]);
    }
    f[4] = 0.5 * ((El + ptl) * vnl - bnl * vbl + (Er + ptr) * vnr - bnr * vbr) - hc * (Er - El);
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        double fl = vnl * wl[5 + q] - bnl * wl[1 + q];
        double fr = vnr * wr[5 + q] - bnr * wr[1 + q];
        if (q == D) {
            fl = 0.0;
            fr = 0.0;
        }
        f[5 + q] = 0.5 * (fl + fr) - hc * (wr[5 + q] - wl[5 + q]);
    }
    if constexpr (NV > 8) f[8] = 0.5 * (ml * wl[8] + mr * wr[8]) - hc * (wr[0] * wr[8] - wl[0] * wl[8]);
}

// Physical ideal-MHD flux of a primitive state along D: rho v_n, rho v_n v -
// B_n B + p_tot e_n, (E + p_tot) v_n - B_n (v.B), v_n B - B_n v (B_n part 0),
// and rho v_n s for the tracer.
template <int D, int NV = 8>
DEV void phys_flux(const double *w, double *f, const Gas &gs)
{
    const double v2 = w[1] * w[1] + w[2] * w[2] + w[3] * w[3];
    const double b2 = w[5] * w[5] + w[6] * w[6] + w[7] * w[7];
    const double pt = w[4] + 0.5 * b2;
    const double E = w[4] * gs.igm1 + 0.5 * w[0] * v2 + 0.5 * b2;
    const double vn = w[1 + D], bn = w[5 + D];
    const double vb = w[1] * w[5] + w[2] * w[6] + w[3] * w[7];
    const double m = w[0] * vn;
    f[0] = m;
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        f[1 + q] = m * w[1 + q] - bn * w[5 + q] + (q == D ? pt : 0.0);
        f[5 + q] = q == D ? 0.0 : vn * w[5 + q] - bn * w[1 + q];
    }
    f[4] = (E + pt) * vn - bn * vb;
    if constexpr (NV > 8) f[8] = m * w[8];
}

// Monotonised-central slope on a non-uniform coordinate (reciprocal spacings given).
DEV double mc_slope(double wm, double w0, double wp, double idm, double idp, double idc)
{
    const double dm = (w0 - wm) * idm;
    const double dp = (wp - w0) * idp;
    const double dc = (wp - wm) * idc;
    const double a = fmin(fabs(dc), 2.0 * fmin(fabs(dm), fabs(dp)));
    return (dm * dp <= 0.0) ? 0.0 : copysign(a, dc);
}

// Limiters of the reconstruction (the paper's runs use the monotonised-central
// "Woodward" form; its code offers others): zero where the one-sided
// differences differ in sign or one vanishes, else LIM_MINMOD the one of
// smaller magnitude, LIM_VANLEER their harmonic mean 2 dm dp / (dm + dp).
enum { LIM_MC = 0, LIM_MINMOD = 1, LIM_VANLEER = 2 };

template <int LIM>
DEV double limited_slope(double wm, double w0, double wp, double idm, double idp, double idc)
{
    if (LIM == LIM_MC) return mc_slope(wm, w0, wp, idm, idp, idc);
    const double dm = (w0 - wm) * idm;
    const double dp = (wp - w0) * idp;
    double sl;
    if (LIM == LIM_MINMOD) sl = fabs(dm) < fabs(dp) ? dm : dp;
    else sl = 2.0 * dm * dp * IC_RCP(dm + dp);
    return (dm * dp <= 0.0) ? 0.0 : sl;
}

// Face values of a cell from its neighbours along one direction; falls back to
// zero slope for all variables if a face density or pressure is not positive.
template <int LIM = LIM_MC, int NV = 8>
DEV void reconstruct(const double *wm, const double *w0, const double *wp, double idm,
                     double idp, double idc, double hm, double hp, double *lo, double *hi)
{
    double s[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) s[v] = limited_slope<LIM>(wm[v], w0[v], wp[v], idm, idp, idc);
    // the density and pressure face values decide; a zero slope gives w0 - 0 * h = w0 exactly
    const bool ok = w0[0] - s[0] * hm > 0.0 && w0[0] + s[0] * hp > 0.0 && w0[4] - s[4] * hm > 0.0 &&
                    w0[4] + s[4] * hp > 0.0;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double sv = ok ? s[v] : 0.0;
        lo[v] = w0[v] - sv * hm;
        hi[v] = w0[v] + sv * hp;
    }
}

// Geometric (hoop), frame (Coriolis, centrifugal) and gravity sources of a
// cell in spherical geometry, added to acc.
DEV void add_sources(const double w[8], double rt, double ctil, double rc, double sc, double cc,
                     double om, double gm, double acc[8])
{
    const double rho = w[0], vr = w[1], vt = w[2], vp = w[3];
    const double br = w[5], bt = w[6], bp = w[7];
    const double ptot = w[4] + 0.5 * (br * br + bt * bt + bp * bp);
    const double g = -gm * IC_RCP(rc * rc);
    acc[1] += rt * (rho * (vt * vt + vp * vp) - (bt * bt + bp * bp) + 2.0 * ptot)
              + rho * (2.0 * om * sc * vp + om * om * rc * sc * sc) + rho * g;
    acc[2] += rt * (-(rho * vr * vt - br * bt) + ctil * (rho * vp * vp - bp * bp + ptot))
              + rho * (2.0 * om * cc * vp + om * om * rc * sc * cc);
    acc[3] += -rt * ((rho * vp * vr - bp * br) + ctil * (rho * vp * vt - bp * bt))
              - 2.0 * om * rho * (sc * vr + cc * vt);
    acc[4] += rho * vr * g + rho * om * om * rc * sc * (vr * sc + vt * cc);
    acc[6] += rt * (vr * bt - vt * br);
    acc[7] += -rt * ((vp * br - bp * vr) + ctil * (vp * bt - bp * vt));
}

// Small-value floors on a conserved state: density first (a cell below the
// density floor takes it at zero velocity), then pressure (energy raised); the
// tracer's rho s is left as it is.  Returns which floors acted: bit 0
// density, bit 1 pressure.
DEV int apply_floors(double u[8], const Gas &gs, double rho_min, double p_min)
{
    int fired = 0;
    if (u[0] < rho_min) {
        u[0] = rho_min;
        u[1] = 0.0;
        u[2] = 0.0;
        u[3] = 0.0;
        fired = 1;
    }
    const double kin = 0.5 * (u[1] * u[1] + u[2] * u[2] + u[3] * u[3]) * IC_RCP(u[0]);
    const double mag = 0.5 * (u[5] * u[5] + u[6] * u[6] + u[7] * u[7]);
    const double p = gs.gm1 * (u[4] - kin - mag);
    if (p < p_min) {
        u[4] = p_min * gs.igm1 + kin + mag;
        fired |= 2;
    }
    return fired;
}
