// kernels.hip -- HIP kernels of the Icarus hot path around the stage kernel
// (gfx950): ghost slabs (inner boundary, restriction, prolongation), reflux,
// CFL rates and the time step, the refinement indicator, regrid data moves
// and point sampling.  The fused stage kernel is in stage.hip.
#include "common.h"

// ---------------------------------------------------------------------------
// Limited linear prolongation from one coarse cell to its 8 children: local
// index cl in the ghosted source block src, wrapped global index cw on level
// geometry cg; the children sit on level geometry lg from the (even,
// unwrapped) global fine index g0 on.  Slopes are minmod of the one-sided
// coordinate differences, applied about the volume centroid of the two
// children along each direction.  A coarse cell whose linear values would
// give any child rho <= 0 or p <= 0 hands its own value to all of them
// (conservative either way).  value(o, v): child o = ox + 2 oy + 4 oz.
template <int NV>
struct Prolong {
    double uc[NV], sl[3][NV], off[3][2];
    bool ok;
    DEV double linear(int o, int v) const
    {
        double x = uc[v];
        x += sl[0][v] * off[0][o & 1];
        x += sl[1][v] * off[1][(o >> 1) & 1];
        x += sl[2][v] * off[2][(o >> 2) & 1];
        return x;
    }
    DEV double value(int o, int v) const { return ok ? linear(o, v) : uc[v]; }
};

template <int BI, int BJ, int BK, int NV>
DEV void prolong_setup(const KArgs &a, int src, const int cl[3], const int cw[3], const LevelGeo &cg,
                       const LevelGeo &lg, const int g0[3], Prolong<NV> &P)
{
    using S = Shape<BI, BJ, BK, NV>;
    const double idm[3] = {cg.r[cw[0] + 2].idm, cg.t[cw[1] + 2].idm, cg.p[cw[2] + 2].idm};
    const double idp[3] = {cg.r[cw[0] + 2].idp, cg.t[cw[1] + 2].idp, cg.p[cw[2] + 2].idp};
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        P.uc[v] = ghosted<S>(a.U, a.desc, a.slabs, a.slab_stride, src, v, cl[0], cl[1], cl[2]);
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            int lm[3] = {cl[0], cl[1], cl[2]}, lp[3] = {cl[0], cl[1], cl[2]};
            lm[e] -= 1;
            lp[e] += 1;
            const double um = ghosted<S>(a.U, a.desc, a.slabs, a.slab_stride, src, v, lm[0], lm[1], lm[2]);
            const double up = ghosted<S>(a.U, a.desc, a.slabs, a.slab_stride, src, v, lp[0], lp[1], lp[2]);
            const double sa = (P.uc[v] - um) * idm[e], sb = (up - P.uc[v]) * idp[e];
            P.sl[e][v] = sa * sb > 0.0 ? copysign(fmin(fabs(sa), fabs(sb)), sa) : 0.0;
        }
    }
#pragma unroll
    for (int o = 0; o < 2; ++o) {
        P.off[0][o] = lg.r[g0[0] + o + 2].poff;
        P.off[1][o] = lg.t[g0[1] + o + 2].poff;
        P.off[2][o] = lg.p[g0[2] + o + 2].poff;
    }
    bool ok = true;
    for (int o = 0; o < 8; ++o) {
        double c[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) c[v] = P.linear(o, v);
        const double kin = 0.5 * (c[1] * c[1] + c[2] * c[2] + c[3] * c[3]) / c[0];
        const double mag = 0.5 * (c[5] * c[5] + c[6] * c[6] + c[7] * c[7]);
        ok = ok && c[0] > 0.0 && c[4] - kin - mag > 0.0;
    }
    P.ok = ok;
}

// ---------------------------------------------------------------------------
// ghost slabs: inner boundary (wind + cone CME), restriction, prolongation
// ---------------------------------------------------------------------------
// Slab tasks whose face is normal to direction D (a template parameter, so
// that every per-direction index below is a register, not private memory).
// Slab layout: element ((v * 2 + l) * FB + b) * FA + a, layer l = 0 nearest
// the low side.
//
// Prolongation slab, one coarse parent cell c (HA x HB parents behind the
// face): the parent's value and minmod slopes along r, theta, phi per
// variable; if the linear values give all 8 children (2 layers x 2 x 2 fine
// cells) rho > 0 and p > 0 they take them, else the parent's own value (the
// prolongation stays conservative either way).
template <int BI, int BJ, int BK, int NV, int D>
DEV void prolong_parent(const KArgs &a, const SlabTask *tkp, int c)
{
    using S = Shape<BI, BJ, BK, NV>;
    constexpr int E1 = tan1(D), E2 = tan2(D);
    constexpr int FA = S::dim(E1), FB = S::dim(E2), Bd = S::dim(D);
    constexpr int HA = FA / 2;
    const int side = tkp->face & 1;
    const BlockDesc bd = a.desc[tkp->slot];
    const LevelGeo lg = a.geo[bd.level];
    const LevelGeo cg = a.geo[bd.level - 1];
    double *out = a.slabs + (size_t)tkp->slab * a.slab_stride;
    const int g0d = side ? bd.org[D] + Bd : bd.org[D] - 2;     // owner-level index of layer 0 along D
    const int cs = tkp->src[0];
    const Faces cnb = load_faces(a.desc, cs);       // the coarse parent block's face codes
    const int pa = c % HA, pb = c / HA;
    int g0[3];                                      // the first child, owner-level global index
    g0[D] = g0d;
    g0[E1] = bd.org[E1] + 2 * pa;
    g0[E2] = bd.org[E2] + 2 * pb;
    int cl[3], cw[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
        const int c2 = g0[e] >= 0 ? g0[e] / 2 : -((-g0[e] + 1) / 2);   // floor(g/2)
        cl[e] = c2 + tkp->shift[e];
        cw[e] = c2 + tkp->cwrap[e];
    }
    const double idm[3] = {cg.r[cw[0] + 2].idm, cg.t[cw[1] + 2].idm, cg.p[cw[2] + 2].idm};
    const double idp[3] = {cg.r[cw[0] + 2].idp, cg.t[cw[1] + 2].idp, cg.p[cw[2] + 2].idp};
    // the children's offsets from the parent's centre, two per direction
    const double off[3][2] = {{lg.r[g0[0] + 2].poff, lg.r[g0[0] + 3].poff},
                              {lg.t[g0[1] + 2].poff, lg.t[g0[1] + 3].poff},
                              {lg.p[g0[2] + 2].poff, lg.p[g0[2] + 3].poff}};
    double P[NV][4];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const double uc = *cell_addr<S>(a.U, a.slabs, a.slab_stride, cs, cnb, v, cl[0], cl[1], cl[2]);
        P[v][0] = uc;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            int lm[3] = {cl[0], cl[1], cl[2]}, lp[3] = {cl[0], cl[1], cl[2]};
            lm[e] -= 1;
            lp[e] += 1;
            const double um = *cell_addr<S>(a.U, a.slabs, a.slab_stride, cs, cnb, v, lm[0], lm[1], lm[2]);
            const double up = *cell_addr<S>(a.U, a.slabs, a.slab_stride, cs, cnb, v, lp[0], lp[1], lp[2]);
            const double sa = (uc - um) * idm[e], sb = (up - uc) * idp[e];
            P[v][1 + e] = sa * sb > 0.0 ? copysign(fmin(fabs(sa), fabs(sb)), sa) : 0.0;
        }
    }
    bool ok = true;
#pragma unroll
    for (int o = 0; o < 8; ++o) {
        double q[8];
#pragma unroll
        for (int v = 0; v < 8; ++v) {
            double x = P[v][0];
            x += P[v][1] * off[0][o & 1];
            x += P[v][2] * off[1][(o >> 1) & 1];
            x += P[v][3] * off[2][(o >> 2) & 1];
            q[v] = x;
        }
        const double kin = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
        const double mag = 0.5 * (q[5] * q[5] + q[6] * q[6] + q[7] * q[7]);
        ok = ok && q[0] > 0.0 && q[4] - kin - mag > 0.0;
    }
    // the children, a pair along E1 (adjacent, 16-byte aligned: even index,
    // even face width) per store
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int l = 0; l < 2; ++l)
#pragma unroll
            for (int hb = 0; hb < 2; ++hb) {
                double x[2];
#pragma unroll
                for (int ha = 0; ha < 2; ++ha) {
                    int h[3];                       // the child's half along each direction
                    h[D] = l;
                    h[E1] = ha;
                    h[E2] = hb;
                    x[ha] = P[v][0];
                    if (ok) {
                        x[ha] += P[v][1] * off[0][h[0]];
                        x[ha] += P[v][2] * off[1][h[1]];
                        x[ha] += P[v][3] * off[2][h[2]];
                    }
                }
                const int ib = 2 * pb + hb;
                *reinterpret_cast<double2 *>(out + ((size_t)(v * 2 + l) * FB + ib) * FA + 2 * pa) =
                    make_double2(x[0], x[1]);
            }
}

// Inner-boundary or restriction slab task, elements part, part + nparts, ...
// (in units of the work-group size): a task's elements split over nparts
// work-groups.
template <int BI, int BJ, int BK, int NV, int D>
DEV void slab_task(const KArgs &a, const SlabTask *tkp, int part, int nparts)
{
    using S = Shape<BI, BJ, BK, NV>;
    constexpr int E1 = tan1(D), E2 = tan2(D);
    constexpr int FA = S::dim(E1), FB = S::dim(E2), Bd = S::dim(D);
    constexpr int NCELL = 2 * FA * FB;
    const int type = tkp->type, side = tkp->face & 1;
    const BlockDesc bd = a.desc[tkp->slot];
    const LevelGeo lg = a.geo[bd.level];
    double *out = a.slabs + (size_t)tkp->slab * a.slab_stride;
    const int g0d = side ? bd.org[D] + Bd : bd.org[D] - 2;     // owner-level index of layer 0 along D
    if (type == SLAB_INNER) {
        const Gas gs = a.gas;
        for (int c = part * blockDim.x + threadIdx.x; c < NCELL; c += nparts * blockDim.x) {
            const int ia = c % FA, ib = (c / FA) % FB, l = c / (FA * FB);
            int g[3];                               // owner-level global index (unwrapped)
            g[D] = g0d + l;
            g[E1] = bd.org[E1] + ia;
            g[E2] = bd.org[E2] + ib;
            const int jt = g[1], kp = g[2];
            const int nt = lg.n[1], np = lg.n[2];
            const size_t o = (size_t)jt * np + kp;
            const size_t pl = (size_t)nt * np;
            double w[NV], u[NV];
            w[0] = lg.wind[0 * pl + o];
            w[1] = lg.wind[1 * pl + o];
            w[2] = 0.0;
            w[3] = lg.wind[2 * pl + o];
            w[4] = lg.wind[3 * pl + o];
            w[5] = lg.wind[4 * pl + o];
            w[6] = 0.0;
            w[7] = lg.wind[5 * pl + o];
            if constexpr (NV > 8) w[8] = 0.0;         // tracer: wind material
            const int mem = bd.member;
            const MemberConst mc = a.mc[mem];
            if (mc.enabled) {
                const double ts = a.t[mem] + a.tfrac * a.dt[mem];
                const double tau = ts - mc.t0;
                if (tau >= 0.0 && tau <= mc.tact) {
                    const double R = mc.r_in;
                    const double Rc = tau * mc.v + R - mc.r_half;
                    double arg = (Rc * Rc + R * R - mc.r_half * mc.r_half) / (2.0 * Rc * R);
                    arg = arg > 1.0 ? 1.0 : (arg < -1.0 ? -1.0 : arg);
                    double cd = lg.cosd[(size_t)mem * pl + o];
                    cd = cd > 1.0 ? 1.0 : (cd < -1.0 ? -1.0 : cd);
                    if (cd >= arg) {
                        w[0] = mc.rho;
                        w[1] = mc.v;
                        w[4] = mc.p;
                        if constexpr (NV > 8) w[8] = 1.0;     // CME material
                    }
                }
            }
            prim_to_cons<NV>(w, u, gs);
#pragma unroll
            for (int v = 0; v < NV; ++v) out[((size_t)(v * 2 + l) * FB + ib) * FA + ia] = u[v];
        }
        return;
    }
    // SLAB_RESTRICT: one thread per ghost cell and group of VG variables (the
    // variables in NG groups; the two children along r of each (theta, phi)
    // child pair are adjacent in memory and 16-byte aligned -- even r index,
    // even block dimensions -- so 4 VG independent 16-byte loads, issued
    // together; the sums run over the children in the same order as one by one)
    constexpr int NG = NV % 4 == 0 ? 2 : 3, VG = NV / NG;
    static_assert(NG * VG == NV, "variable groups of the restriction");
    const LevelGeo fg = a.geo[bd.level + 1];
    const int shift[3] = {tkp->shift[0], tkp->shift[1], tkp->shift[2]};
    const int fbase[3] = {tkp->fbase[0], tkp->fbase[1], tkp->fbase[2]};
    const int src0 = tkp->src[0], src1 = tkp->src[1], src2 = tkp->src[2], src3 = tkp->src[3];
    for (int e = part * blockDim.x + threadIdx.x; e < NG * NCELL; e += nparts * blockDim.x) {
        const int c = e % NCELL, h = e / NCELL;
        // along r the two layers of a ghost cell go to adjacent lanes: their
        // children are the four fine r-cells of one row, contiguous in memory;
        // across r, lanes follow the slab (the children rows run along r)
        const int ia = D == 0 ? (c >> 1) % FA : c % FA;
        const int ib = D == 0 ? (c >> 1) / FA : (c / FA) % FB;
        const int l = D == 0 ? c & 1 : c / (FA * FB);
        int gw[3];                                  // owner-level global index, wrapped
        gw[D] = g0d + l + shift[D];
        gw[E1] = bd.org[E1] + ia + shift[E1];
        gw[E2] = bd.org[E2] + ib + shift[E2];
        // volume factors of the two children along each direction
        const double wr[2] = {fg.r[2 * gw[0] + 2].vw, fg.r[2 * gw[0] + 3].vw};
        const double wt[2] = {fg.t[2 * gw[1] + 2].vw, fg.t[2 * gw[1] + 3].vw};
        const double wp[2] = {fg.p[2 * gw[2] + 2].vw, fg.p[2 * gw[2] + 3].vw};
        double num[VG], den = 0.0;
#pragma unroll
        for (int v = 0; v < VG; ++v) num[v] = 0.0;
#pragma unroll
        for (int o2 = 0; o2 < 4; ++o2) {            // children o = 2 o2 and 2 o2 + 1 (r offset 0, 1)
            int fl[3], q[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int fgi = 2 * gw[d] + (d == 0 ? 0 : (o2 >> (d - 1)) & 1);
                const int fb = fgi / S::dim(d);
                q[d] = fb - fbase[d];
                fl[d] = fgi - fb * S::dim(d);
            }
            const int qq = q[E1] + 2 * q[E2];
            const int fslot = qq == 0 ? src0 : (qq == 1 ? src1 : (qq == 2 ? src2 : src3));
            const double wgt0 = wr[0] * wt[o2 & 1] * wp[(o2 >> 1) & 1];
            const double wgt1 = wr[1] * wt[o2 & 1] * wp[(o2 >> 1) & 1];
            double2 x[VG];
#pragma unroll
            for (int v = 0; v < VG; ++v)
                x[v] = *reinterpret_cast<const double2 *>(a.U + cidx<S>(fslot, VG * h + v, fl[0], fl[1], fl[2]));
#pragma unroll
            for (int v = 0; v < VG; ++v) num[v] += wgt0 * x[v].x;
            den += wgt0;
#pragma unroll
            for (int v = 0; v < VG; ++v) num[v] += wgt1 * x[v].y;
            den += wgt1;
        }
#pragma unroll
        for (int v = 0; v < VG; ++v) out[((size_t)((VG * h + v) * 2 + l) * FB + ib) * FA + ia] = num[v] / den;
    }
}

// PASS 0: inner-boundary and restriction slabs, each task's elements split
// over SLAB_PARTS work-groups (a pass of few tasks then spreads over more
// compute units, and each work-group's chain of dependent loads is shorter);
// PASS 1: prolongation slabs, one wave per task and one lane per coarse
// parent (at most 64 per face), so no task waits on a barrier (separate
// kernels, so that each is compiled for its own register needs)
constexpr int SLAB_PARTS = 3;
constexpr int PROLONG_TASKS = NT / 64;          // prolongation tasks per work-group

template <int BI, int BJ, int BK, int NV, int PASS>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(PASS == 1 ? 2 : 1)))
k_slabs(KArgs a, const SlabTask *tasks, const int *range)
{
    using S = Shape<BI, BJ, BK, NV>;
    const int t0 = range[0], t1 = range[1];
    if (PASS == 1) {
        static_assert(S::MAXFACE / 4 <= 64, "coarse parents of a face per wave");
        const int lane = threadIdx.x % 64;
        for (int it = t0 + blockIdx.x * PROLONG_TASKS + threadIdx.x / 64; it < t1; it += gridDim.x * PROLONG_TASKS) {
            const int d = tasks[it].face >> 1;      // uniform over the wave
            if (d == 0) {
                if (lane < S::face_cells(0) / 4) prolong_parent<BI, BJ, BK, NV, 0>(a, tasks + it, lane);
            } else if (d == 1) {
                if (lane < S::face_cells(1) / 4) prolong_parent<BI, BJ, BK, NV, 1>(a, tasks + it, lane);
            } else if (lane < S::face_cells(2) / 4) {
                prolong_parent<BI, BJ, BK, NV, 2>(a, tasks + it, lane);
            }
        }
        return;
    }
    const int nu = (t1 - t0) * SLAB_PARTS;
    for (int u = blockIdx.x; u < nu; u += gridDim.x) {
        const int it = t0 + u / SLAB_PARTS, part = u % SLAB_PARTS;
        const int d = tasks[it].face >> 1;          // uniform over the work-group
        if (d == 0) slab_task<BI, BJ, BK, NV, 0>(a, tasks + it, part, SLAB_PARTS);
        else if (d == 1) slab_task<BI, BJ, BK, NV, 1>(a, tasks + it, part, SLAB_PARTS);
        else slab_task<BI, BJ, BK, NV, 2>(a, tasks + it, part, SLAB_PARTS);
    }
}

// ---------------------------------------------------------------------------
// reflux at coarse-fine faces, then the CFL rates of the corrected cells
// ---------------------------------------------------------------------------
// (the 8 MHD variables of u are read)
__device__ inline double cell_rate(const double *u, const RecR &rr, const RecT &tt, const RecP &pp, const Gas &gs)
{
    double w[8];
    cons_to_prim(u, w, gs);
    return (fabs(w[1]) + fast_speed<0>(w, gs)) * rr.icfl
         + (fabs(w[2]) + fast_speed<1>(w, gs)) * rr.irc * tt.icfl
         + (fabs(w[3]) + fast_speed<2>(w, gs)) * rr.irc * tt.isinc * pp.iw;
}

// Reflux correction of one coarse cell (loc, block coordinates) behind the
// coarse-fine face of task tk, face direction D (a template parameter: every
// per-direction index stays in registers): (A_c F_c - sum of the 4 fine A F)
// / V_c per variable, the fine faces summed in fixed order.
template <int BI, int BJ, int BK, int NV, int D>
DEV void reflux_corr(const KArgs &a, const RefluxTask &tk, const BlockDesc &bd, const LevelGeo &lg,
                     const LevelGeo &fg, const int loc[3], double corr[NV])
{
    using S = Shape<BI, BJ, BK, NV>;
    constexpr int E1 = tan1(D), E2 = tan2(D);
    constexpr int FA = S::dim(E1), FB = S::dim(E2);
    const int side = tk.face & 1;
    const int ia = loc[E1], ib = loc[E2];
    int g[3];
#pragma unroll
    for (int e = 0; e < 3; ++e) g[e] = bd.org[e] + loc[e];
    const RecR rr = lg.r[g[0] + 2];
    const RecT tt = lg.t[g[1] + 2];
    const RecP pp = lg.p[g[2] + 2];
    const double Vc = rr.vw * tt.vw * pp.vw;
    double ac;
    if (D == 0) ac = side ? rr.ap : rr.am;
    else if (D == 1) ac = rr.rt * (side ? tt.thp : tt.thm);
    else ac = rr.rt * tt.phf * pp.iw;
    const int gf = 2 * (bd.org[D] + (side ? S::dim(D) : 0));   // fine face index along D
    const double *Fc = a.freg + (size_t)tk.creg * a.reg_stride;
    double sum[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) sum[v] = 0.0;
#pragma unroll
    for (int ob = 0; ob < 2; ++ob) {
#pragma unroll
        for (int oa = 0; oa < 2; ++oa) {
            const int fa = 2 * ia + oa, fb = 2 * ib + ob;
            const int qa = fa / FA, qb = fb / FB;
            const int qq = qa + 2 * qb;
            const int reg = qq == 0 ? tk.freg[0] : (qq == 1 ? tk.freg[1] : (qq == 2 ? tk.freg[2] : tk.freg[3]));
            int fgl[3];
            fgl[D] = gf;
            fgl[E1] = 2 * g[E1] + oa;
            fgl[E2] = 2 * g[E2] + ob;
            double A;
            if (D == 0) A = fg.r[fgl[0] + 2].r2f * fg.t[fgl[1] + 2].vw * fg.p[fgl[2] + 2].vw;
            else if (D == 1) A = fg.r[fgl[0] + 2].r2h * fg.t[fgl[1] + 2].sf * fg.p[fgl[2] + 2].vw;
            else A = fg.r[fgl[0] + 2].r2h * fg.t[fgl[1] + 2].dth;
            const double *F = a.freg + (size_t)reg * a.reg_stride;
            const int la = fa - qa * FA, lb = fb - qb * FB;
#pragma unroll
            for (int v = 0; v < NV; ++v) sum[v] += A * F[((size_t)v * FB + lb) * FA + la];
        }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) corr[v] = ac * Fc[((size_t)v * FB + ib) * FA + ia] - sum[v] / Vc;
}

// Is cell (i, j, k) on face f (2 d + side) of its block?
template <int BI, int BJ, int BK>
DEV bool on_face(int f, int i, int j, int k)
{
    const int d = f >> 1;
    const int x = d == 0 ? i : (d == 1 ? j : k);
    const int n = d == 0 ? BI : (d == 1 ? BJ : BK);
    return x == ((f & 1) ? n - 1 : 0);
}

// One work-group per reflux task (a coarse-fine face of a coarse block; the
// block's tasks are ranges[2q] .. ranges[2q+1], in face order).  Each cell
// behind the face takes U += +-adt (A_c F_c - sum A F) / V_c; a cell on
// several of the block's reflux faces (an edge or corner) is corrected by the
// work-group of the last of them, face by face in task order, so every cell
// has one writer and the corrections add in the same order as face after
// face.  Then the floors and the CFL rate of each corrected cell (the stage
// kernel left these cells out of its maxima), folded into the block's entry.
template <int BI, int BJ, int BK, int NV>
__global__ void __launch_bounds__(NT) k_reflux(KArgs a, const RefluxTask *tasks, const int *ranges, const int *ntasks)
{
    using S = Shape<BI, BJ, BK, NV>;
    __shared__ double sred[NT / 64];
    const int nt = *ntasks;
    for (int q = blockIdx.x; q < nt; q += gridDim.x) {
        const int t0 = ranges[2 * q], t1 = ranges[2 * q + 1];
        const int slot = tasks[q].slot;
        const BlockDesc bd = a.desc[slot];
        const double dt = a.dt[bd.member];
        if (dt <= 0.0) continue;                    // uniform over the work-group
        const double adt = a.alpha * dt;
        const LevelGeo lg = a.geo[bd.level], fg = a.geo[bd.level + 1];
        // the block's reflux faces in task order, 3 bits each (at most 6)
        const int nf = t1 - t0, me = q - t0;
        unsigned fc = 0;
        for (int p = 0; p < nf; ++p) fc |= (unsigned)tasks[t0 + p].face << (3 * p);
        const int d = tasks[q].face >> 1, side = tasks[q].face & 1;
        double rmax = 0.0;
        int badc = -1, nfr = 0, nfp = 0;
        for (int c = threadIdx.x; c < S::face_cells(d); c += blockDim.x) {
            int i, j, k;                            // the cell: index c on face (d, side)
            if (d == 0) i = side ? BI - 1 : 0, j = c % BJ, k = c / BJ;
            else if (d == 1) i = c % BI, j = side ? BJ - 1 : 0, k = c / BI;
            else i = c % BI, j = c / BI, k = side ? BK - 1 : 0;
            bool last = true;
            for (int p = me + 1; p < nf; ++p)
                if (on_face<BI, BJ, BK>((fc >> (3 * p)) & 7, i, j, k)) last = false;
            if (!last) continue;
            double u[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) u[v] = a.Uout[cidx<S>(slot, v, i, j, k)];
            const int loc[3] = {i, j, k};
            for (int p = 0; p <= me; ++p) {
                const int fp = (fc >> (3 * p)) & 7;
                if (!on_face<BI, BJ, BK>(fp, i, j, k)) continue;
                const RefluxTask tk = tasks[t0 + p];
                double corr[NV];
                const int dp = fp >> 1;
                if (dp == 0) reflux_corr<BI, BJ, BK, NV, 0>(a, tk, bd, lg, fg, loc, corr);
                else if (dp == 1) reflux_corr<BI, BJ, BK, NV, 1>(a, tk, bd, lg, fg, loc, corr);
                else reflux_corr<BI, BJ, BK, NV, 2>(a, tk, bd, lg, fg, loc, corr);
                const int sp = fp & 1;
#pragma unroll
                for (int v = 0; v < NV; ++v) u[v] += sp ? adt * corr[v] : -adt * corr[v];
            }
            const int f = apply_floors(u, a.gas, a.rho_floor, a.p_floor);
            nfr += f & 1;
            nfp += f >> 1;
#pragma unroll
            for (int v = 0; v < NV; ++v) a.Uout[cidx<S>(slot, v, i, j, k)] = u[v];
            if (a.want_rate) {
                double w[NV];
                cons_to_prim<false, NV>(u, w, a.gas);
                if (badc < 0 && unphysical<NV>(w)) badc = i + BI * (j + BJ * k);
                const double r = cell_rate(u, lg.r[bd.org[0] + i + 2], lg.t[bd.org[1] + j + 2],
                                                       lg.p[bd.org[2] + k + 2], a.gas);
                rmax = r > rmax ? r : rmax;
            }
        }
        if (badc >= 0 && atomicCAS(&a.bad[2 * bd.member], 0, slot + 1) == 0) a.bad[2 * bd.member + 1] = badc;
        if (nfr | nfp) {
            atomicAdd(&a.floors[2 * bd.member], (unsigned long long)nfr);
            atomicAdd(&a.floors[2 * bd.member + 1], (unsigned long long)nfp);
        }
        if (a.want_rate) {
            // the block's other faces may fold theirs in concurrently: rates are
            // >= 0 and not NaN (a NaN rate fails the comparisons above), so the
            // unsigned order of their bits is their numeric order
            const double m = block_max(rmax, sred);
            if (threadIdx.x == 0)
                atomicMax((unsigned long long *)&a.rate[(size_t)slot * KSPLIT_MAX],
                          (unsigned long long)__double_as_longlong(m));
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Hancock predictor (the one-step TVDLF form): U* = U + alpha dt L_H(U), L_H
// the finite-volume difference of each cell's own physical fluxes at its
// reconstructed lower and upper face states, plus the sources at the cell
// state; no interface solver and no reflux (the corrector, a stage-kernel
// launch from U*, is conservative).  One work-group per leaf block, one
// thread per cell; neighbours along each axis through cell_addr (one index
// at most in the ghost layers).  Floors and the input check as in k_stage.
// ---------------------------------------------------------------------------
template <class S>
DEV void prim_at(const KArgs &a, int slot, const Faces &nb, int i, int j, int k, double *w)
{
    double u[S::NV];
#pragma unroll
    for (int v = 0; v < S::NV; ++v) u[v] = *cell_addr<S>(a.U, a.slabs, a.slab_stride, slot, nb, v, i, j, k);
    cons_to_prim<false, S::NV>(u, w, a.gas);
}

template <int BI, int BJ, int BK, int NV, int LIM>
__global__ void __launch_bounds__(NT) k_hancock(KArgs a)
{
    using S = Shape<BI, BJ, BK, NV>;
    const int n = *a.nitems;
    const Gas gs = a.gas;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int slot = a.items[it];
        const int mem = a.desc[slot].member;
        const double dt = a.dt[mem];
        if (dt <= 0.0) continue;
        const double adt = a.alpha * dt;
        const LevelGeo lg = a.geo[a.desc[slot].level];
        const int o0 = a.desc[slot].org[0], o1 = a.desc[slot].org[1], o2 = a.desc[slot].org[2];
        const Faces nb = load_faces(a.desc, slot);
        int badc = -1, nfr = 0, nfp = 0;
        for (int c = threadIdx.x; c < S::NC; c += NT) {
            const int i = c % BI, j = (c / BI) % BJ, k = c / (BI * BJ);
            double w0[NV], acc[NV];
            prim_at<S>(a, slot, nb, i, j, k, w0);
            if (badc < 0 && unphysical<NV>(w0)) badc = c;
#pragma unroll
            for (int v = 0; v < NV; ++v) acc[v] = 0.0;
            const RecR rr = lg.r[o0 + i + 2];
            const RecT tt = lg.t[o1 + j + 2];
            const RecP pk = lg.p[o2 + k + 2];
            {   // r
                double wm[NV], wp[NV], lo[NV], hi[NV], fl[NV], fh[NV];
                prim_at<S>(a, slot, nb, i - 1, j, k, wm);
                prim_at<S>(a, slot, nb, i + 1, j, k, wp);
                reconstruct<LIM, NV>(wm, w0, wp, rr.idm, rr.idp, rr.idc, rr.hm, rr.hp, lo, hi);
                phys_flux<0, NV>(lo, fl, gs);
                phys_flux<0, NV>(hi, fh, gs);
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] -= rr.ap * fh[v] - rr.am * fl[v];
            }
            {   // theta
                double wm[NV], wp[NV], lo[NV], hi[NV], fl[NV], fh[NV];
                prim_at<S>(a, slot, nb, i, j - 1, k, wm);
                prim_at<S>(a, slot, nb, i, j + 1, k, wp);
                reconstruct<LIM, NV>(wm, w0, wp, tt.idm, tt.idp, tt.idc, tt.hm, tt.hp, lo, hi);
                phys_flux<1, NV>(lo, fl, gs);
                phys_flux<1, NV>(hi, fh, gs);
                const double thm = rr.rt * tt.thm, thp = rr.rt * tt.thp;
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] -= thp * fh[v] - thm * fl[v];
            }
            {   // phi
                double wm[NV], wp[NV], lo[NV], hi[NV], fl[NV], fh[NV];
                prim_at<S>(a, slot, nb, i, j, k - 1, wm);
                prim_at<S>(a, slot, nb, i, j, k + 1, wp);
                reconstruct<LIM, NV>(wm, w0, wp, pk.idm, pk.idp, pk.idc, pk.hm, pk.hp, lo, hi);
                phys_flux<2, NV>(lo, fl, gs);
                phys_flux<2, NV>(hi, fh, gs);
                const double kf = rr.rt * tt.phf * pk.iw;
#pragma unroll
                for (int v = 0; v < NV; ++v) acc[v] -= kf * fh[v] - kf * fl[v];
            }
            if (!a.cart) add_sources(w0, rr.rt, tt.ctil, rr.rc, tt.sinc, tt.cosc, a.omega, a.gm, acc);
            double unew[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) unew[v] = a.Ubase[cidx<S>(slot, v, i, j, k)] + adt * acc[v];
            const int f = apply_floors(unew, gs, a.rho_floor, a.p_floor);
            nfr += f & 1;
            nfp += f >> 1;
#pragma unroll
            for (int v = 0; v < NV; ++v) a.Uout[cidx<S>(slot, v, i, j, k)] = unew[v];
        }
        if (badc >= 0 && atomicCAS(&a.bad[2 * mem], 0, slot + 1) == 0) a.bad[2 * mem + 1] = badc;
        if (nfr | nfp) {
            atomicAdd(&a.floors[2 * mem], (unsigned long long)nfr);
            atomicAdd(&a.floors[2 * mem + 1], (unsigned long long)nfp);
        }
    }
}

// the tracer (NV = 9) with the paper's limiter only
template <int BI, int BJ, int BK, int NV>
void launch_hancock(dim3 g, hipStream_t s, const KArgs &a, int limiter)
{
    if (limiter == LIM_MINMOD) hipLaunchKernelGGL((k_hancock<BI, BJ, BK, NV, LIM_MINMOD>), g, dim3(NT), 0, s, a);
    else if (limiter == LIM_VANLEER) hipLaunchKernelGGL((k_hancock<BI, BJ, BK, NV, LIM_VANLEER>), g, dim3(NT), 0, s, a);
    else hipLaunchKernelGGL((k_hancock<BI, BJ, BK, NV, LIM_MC>), g, dim3(NT), 0, s, a);
}

// ---------------------------------------------------------------------------
// parabolic div B cleaning (a stage option): k_divb forms D = div B of the
// stage input per cell (face-mean form, (1/V) sum_d [A+ Bt+ - A- Bt-], ghosts
// filled); after the stage, its reflux and floors, k_clean moves the stage
// result by dB = alpha C_d h^2 grad D (central differences of D between face
// neighbours in physical components, h^2 = 1 / sum_d dx_d^-2 with the CFL
// widths) and E by B_in . dB.  A neighbour across a block face is read from
// the same-level neighbour block's D; across a boundary or a level change the
// gradient component is zero.  In the second stage k_clean also takes the
// output check and the CFL maxima (the stage and reflux kernels leave them).
// ---------------------------------------------------------------------------
template <int BI, int BJ, int BK, int NV>
__global__ void __launch_bounds__(NT) k_divb(KArgs a)
{
    using S = Shape<BI, BJ, BK, NV>;
    const int n = *a.nitems;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int slot = a.items[it];
        const LevelGeo lg = a.geo[a.desc[slot].level];
        const int o0 = a.desc[slot].org[0], o1 = a.desc[slot].org[1], o2 = a.desc[slot].org[2];
        const Faces nb = load_faces(a.desc, slot);
        for (int c = threadIdx.x; c < S::NC; c += NT) {
            const int i = c % BI, j = (c / BI) % BJ, k = c / (BI * BJ);
            const RecR rr = lg.r[o0 + i + 2];
            const RecT tt = lg.t[o1 + j + 2];
            const RecP pk = lg.p[o2 + k + 2];
            const double *U = a.U;
            const double b0 = *cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 5, i, j, k);
            const double b1 = *cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 6, i, j, k);
            const double b2 = *cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 7, i, j, k);
            const double rl = 0.5 * (*cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 5, i - 1, j, k) + b0);
            const double rh = 0.5 * (b0 + *cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 5, i + 1, j, k));
            const double tl = 0.5 * (*cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 6, i, j - 1, k) + b1);
            const double th = 0.5 * (b1 + *cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 6, i, j + 1, k));
            const double pl = 0.5 * (*cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 7, i, j, k - 1) + b2);
            const double ph = 0.5 * (b2 + *cell_addr<S>(U, a.slabs, a.slab_stride, slot, nb, 7, i, j, k + 1));
            const double kf = rr.rt * tt.phf * pk.iw;
            double dv = rr.ap * rh - rr.am * rl;
            dv += rr.rt * tt.thp * th - rr.rt * tt.thm * tl;
            dv += kf * ph - kf * pl;
            a.divb[(size_t)slot * S::NC + c] = dv;
        }
    }
}

template <int BI, int BJ, int BK, int NV>
__global__ void __launch_bounds__(NT) k_clean(KArgs a)
{
    using S = Shape<BI, BJ, BK, NV>;
    __shared__ double sred[NT / 64];
    const int n = *a.nitems;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int slot = a.items[it];
        const int mem = a.desc[slot].member;
        const double dt = a.dt[mem];
        if (dt <= 0.0) continue;                      // uniform over the work-group
        const LevelGeo lg = a.geo[a.desc[slot].level];
        const int o0 = a.desc[slot].org[0], o1 = a.desc[slot].org[1], o2 = a.desc[slot].org[2];
        const Faces nb = load_faces(a.desc, slot);
        const double coef = a.alpha * a.divb_cd;
        const double *D = a.divb + (size_t)slot * S::NC;
        double rmax = 0.0;
        int badc = -1;
        for (int c = threadIdx.x; c < S::NC; c += NT) {
            const int i = c % BI, j = (c / BI) % BJ, k = c / (BI * BJ);
            const int idx[3] = {i, j, k};
            const RecR rr = lg.r[o0 + i + 2];
            const RecT tt = lg.t[o1 + j + 2];
            const RecP pk = lg.p[o2 + k + 2];
            // D at the two face neighbours along d; NaN-free flag `ok`
            double g[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const int st = d == 0 ? 1 : (d == 1 ? BI : BI * BJ);
                const int Bd = d == 0 ? BI : (d == 1 ? BJ : BK);
                bool ok = true;
                double dm, dp;
                if (idx[d] > 0) dm = D[c - st];
                else {
                    const int code = face_code(nb, 2 * d);
                    ok = ok && code >= 0;
                    dm = code >= 0 ? a.divb[(size_t)code * S::NC + c + (Bd - 1) * st] : 0.0;
                }
                if (idx[d] < Bd - 1) dp = D[c + st];
                else {
                    const int code = face_code(nb, 2 * d + 1);
                    ok = ok && code >= 0;
                    dp = code >= 0 ? a.divb[(size_t)code * S::NC + c - (Bd - 1) * st] : 0.0;
                }
                const double isp = d == 0 ? rr.idc : (d == 1 ? rr.irc * tt.idc : rr.irc * tt.isinc * pk.idc);
                g[d] = ok ? (dp - dm) * isp : 0.0;
            }
            const double ix = rr.icfl, iy = rr.irc * tt.icfl, iz = rr.irc * tt.isinc * pk.iw;
            const double h2 = 1.0 / (ix * ix + iy * iy + iz * iz);
            const double ch = coef * h2;
            const size_t base = cidx<S>(slot, 0, i, j, k);
            double u[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) u[v] = a.Uout[base + (size_t)v * S::NC];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                const double db = ch * g[d];
                u[4] += a.U[base + (size_t)(5 + d) * S::NC] * db;
                u[5 + d] += db;
            }
            a.Uout[base + 4 * (size_t)S::NC] = u[4];
#pragma unroll
            for (int d = 0; d < 3; ++d) a.Uout[base + (size_t)(5 + d) * S::NC] = u[5 + d];
            if (a.want_rate) {
                double w[NV];
                cons_to_prim<false, NV>(u, w, a.gas);
                if (badc < 0 && unphysical<NV>(w)) badc = c;
                const double r = cell_rate(u, rr, tt, pk, a.gas);
                rmax = r > rmax ? r : rmax;
            }
        }
        if (badc >= 0 && atomicCAS(&a.bad[2 * mem], 0, slot + 1) == 0) a.bad[2 * mem + 1] = badc;
        if (a.want_rate) {
            const double m = block_max(rmax, sred);
            if (threadIdx.x < KSPLIT_MAX) a.rate[(size_t)slot * KSPLIT_MAX + threadIdx.x] = threadIdx.x == 0 ? m : 0.0;
        }
    }
}

// CFL rate of every leaf (after create, set_state, regrid)
template <int BI, int BJ, int BK, int NV>
__global__ void __launch_bounds__(NT) k_rate(KArgs a)
{
    using S = Shape<BI, BJ, BK, NV>;
    __shared__ double sred[NT / 64];
    const int n = *a.nitems;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int slot = a.items[it];
        const BlockDesc bd = a.desc[slot];
        const LevelGeo lg = a.geo[bd.level];
        double rmax = 0.0;
        int bad = -1;
        for (int c = threadIdx.x; c < S::NC; c += blockDim.x) {
            const int i = c % BI, j = (c / BI) % BJ, k = c / (BI * BJ);
            double u[NV], w[NV];
            for (int v = 0; v < NV; ++v) u[v] = a.U[cidx<S>(slot, v, i, j, k)];
            cons_to_prim<false, NV>(u, w, a.gas);
            if (bad < 0 && unphysical<NV>(w)) bad = c;
            const double r = cell_rate(u, lg.r[bd.org[0] + i + 2], lg.t[bd.org[1] + j + 2],
                                                   lg.p[bd.org[2] + k + 2], a.gas);
            rmax = r > rmax ? r : rmax;
        }
        if (bad >= 0 && atomicCAS(&a.bad[2 * bd.member], 0, slot + 1) == 0) a.bad[2 * bd.member + 1] = bad;
        const double m = block_max(rmax, sred);
        if (threadIdx.x < KSPLIT_MAX) a.rate[(size_t)slot * KSPLIT_MAX + threadIdx.x] = threadIdx.x == 0 ? m : 0.0;
    }
}

// dt per member = cfl / max rate over its leaves (or a fixed dt), clipped to t_end
__global__ void k_dt(KArgs a, const int *mbeg, const int *mend, int nmembers, double cfl,
                     double dt_fixed, const double *tend, double *dt_last)
{
    __shared__ double sred[NT / 64];
    for (int m = blockIdx.x; m < nmembers; m += gridDim.x) {
        double r = 0.0;
        const int q1 = mend[m];
        // four work items per thread and pass: their slot loads, then their
        // rate loads, are in flight together (the maximum is order-free)
        for (int q0 = mbeg[m] + threadIdx.x; q0 < q1; q0 += 4 * blockDim.x) {
            int sl[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int q = q0 + u * (int)blockDim.x;
                sl[u] = q < q1 ? a.items[q] : -1;
            }
            // every part's entry (a part count changed since the last rate
            // refresh leaves its entries valid: each stage clears the ones
            // beyond its own parts), two per 16-byte load
            static_assert(KSPLIT_MAX % 2 == 0, "rate entries in pairs");
#pragma unroll
            for (int u = 0; u < 4; ++u)
                if (sl[u] >= 0) {
                    const double2 *rp = (const double2 *)(a.rate + (size_t)sl[u] * KSPLIT_MAX);
#pragma unroll
                    for (int p = 0; p < KSPLIT_MAX / 2; ++p) {
                        const double2 x = rp[p];
                        r = x.x > r ? x.x : r;
                        r = x.y > r ? x.y : r;
                    }
                }
        }
        const double mx = block_max(r, sred);
        if (threadIdx.x == 0) {
            double dt = dt_fixed > 0.0 ? dt_fixed : (mx > 0.0 ? cfl / mx : 0.0);
            const double left = tend[m] - a.t[m];
            if (dt > left) dt = left;
            if (!(dt > 0.0)) dt = 0.0;
            ((double *)a.dt)[m] = dt;
            if (dt > 0.0) dt_last[m] = dt;
        }
    }
}

__global__ void k_time(double *t, const double *dt, long *nsteps, int nmembers)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m < nmembers && dt[m] > 0.0) {
        t[m] += dt[m];
        nsteps[m] += 1;
    }
}

// ---------------------------------------------------------------------------
// refinement indicator: Loehner(rho, |v|) with div V < 0 inside the windows
// (shock criterion); the tracer fraction s = (rho s) / rho above a threshold
// anywhere (tracer criterion); or either inside the windows (combined)
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
template <int BI, int BJ, int BK, int NV>
__global__ void __launch_bounds__(NT) k_indicator(KArgs a, int8_t *flags, IndicatorParams p)
{
    using S = Shape<BI, BJ, BK, NV>;
    const int max_level = p.max_level, use_windows = p.use_windows;
    const double eps = p.eps, tol_r = p.tol_r, tol_c = p.tol_c, w_rho = p.w_rho, w_v = p.w_v;
    const double lon_e = p.lon_e, clt_e = p.clt_e, dlon_e = p.dlon_e, dclt_e = p.dclt_e, dlon_c = p.dlon_c;
    const int crit = NV > 8 ? p.criterion : CRIT_SHOCK;
    const int n = *a.nitems;
    const double PI = 3.14159265358979323846;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int slot = a.items[it];
        const BlockDesc bd = a.desc[slot];
        const Faces nb = load_faces(a.desc, slot);
        auto cell8 = [&](int i, int j, int k, double u[8]) {
#pragma unroll
            for (int v = 0; v < 8; ++v) u[v] = *cell_addr<S>(a.U, a.slabs, a.slab_stride, slot, nb, v, i, j, k);
        };
        const LevelGeo lg = a.geo[bd.level];
        const double lon_c = a.mc[bd.member].lon_cme;
        const int cme_on = a.mc[bd.member].enabled;
        int hot_r = 0, hot_c = 0;
        for (int c = threadIdx.x; c < S::NC; c += blockDim.x) {
            const int ijk[3] = {c % BI, (c / BI) % BJ, c / (BI * BJ)};
            const RecR rr = lg.r[bd.org[0] + ijk[0] + 2];
            const RecT tt = lg.t[bd.org[1] + ijk[1] + 2];
            const RecP pp = lg.p[bd.org[2] + ijk[2] + 2];
            bool win = true;
            if (use_windows && !a.cart) {
                auto wrap = [&](double x) {
                    double y = x - 2.0 * PI * floor((x + PI) / (2.0 * PI));
                    return y == -PI ? PI : y;
                };
                win = fabs(wrap(pp.pc - lon_e)) <= dlon_e && fabs(tt.tc - clt_e) <= dclt_e;
                if (cme_on) win = win && fabs(wrap(pp.pc - lon_c)) <= dlon_c;
            }
            double u[8], w0[8];
            cell8(ijk[0], ijk[1], ijk[2], u);
            cons_to_prim<true>(u, w0, a.gas);
            // tracer condition on the correctly rounded fraction (rho s) / rho
            bool tr_r = false, tr_c = false;
            if constexpr (NV > 8) {
                if (crit != CRIT_SHOCK) {
                    const double sf = *cell_addr<S>(a.U, a.slabs, a.slab_stride, slot, nb, 8, ijk[0], ijk[1], ijk[2]) / u[0];
                    tr_r = sf > p.tr_r;
                    tr_c = sf > p.tr_c;
                }
            }
            const double r0 = w0[0];
            const double s0 = sqrt(w0[1] * w0[1] + w0[2] * w0[2] + w0[3] * w0[3]);
            double num_r = 0, den_r = 0, num_v = 0, den_v = 0, dv = 0;
            for (int d = 0; d < 3; ++d) {
                int lo[3] = {ijk[0], ijk[1], ijk[2]}, hi[3] = {ijk[0], ijk[1], ijk[2]};
                lo[d] -= 1;
                hi[d] += 1;
                double wl[8], wh[8];
                cell8(lo[0], lo[1], lo[2], u);
                cons_to_prim<true>(u, wl, a.gas);
                cell8(hi[0], hi[1], hi[2], u);
                cons_to_prim<true>(u, wh, a.gas);
                const double rl = wl[0], rh = wh[0];
                const double sl = sqrt(wl[1] * wl[1] + wl[2] * wl[2] + wl[3] * wl[3]);
                const double sh = sqrt(wh[1] * wh[1] + wh[2] * wh[2] + wh[3] * wh[3]);
                double q = rh - 2.0 * r0 + rl;
                num_r += q * q;
                q = fabs(rh - r0) + fabs(r0 - rl) + eps * (fabs(rh) + 2.0 * fabs(r0) + fabs(rl));
                den_r += q * q;
                q = sh - 2.0 * s0 + sl;
                num_v += q * q;
                q = fabs(sh - s0) + fabs(s0 - sl) + eps * (fabs(sh) + 2.0 * fabs(s0) + fabs(sl));
                den_v += q * q;
                const double vl = 0.5 * (wl[1 + d] + w0[1 + d]);
                const double vh = 0.5 * (w0[1 + d] + wh[1 + d]);
                double am, ap;
                if (d == 0) { am = rr.am; ap = rr.ap; }
                else if (d == 1) { am = rr.rt * tt.thm; ap = rr.rt * tt.thp; }
                else { am = ap = rr.rt * tt.phf * pp.iw; }
                dv += ap * vh - am * vl;
            }
            const double E = w_rho * (den_r > 0.0 ? sqrt(num_r / den_r) : 0.0)
                           + w_v * (den_v > 0.0 ? sqrt(num_v / den_v) : 0.0);
            if (crit == CRIT_TRACER) {
                if (tr_r) hot_r = 1;
                if (tr_c) hot_c = 1;
            } else {
                if (win && dv < 0.0) {
                    if (E > tol_r) hot_r = 1;
                    if (E > tol_c) hot_c = 1;
                }
                if (crit == CRIT_COMBINED && win) {
                    if (tr_r) hot_r = 1;
                    if (tr_c) hot_c = 1;
                }
            }
        }
        hot_r = __syncthreads_or(hot_r);
        hot_c = __syncthreads_or(hot_c);
        if (threadIdx.x == 0) {
            int8_t f = 0;
            if (bd.level < max_level && hot_r) f = 1;
            else if (bd.level > 1 && !hot_c) f = -1;
            flags[slot] = f;
        }
    }
}
#pragma clang fp contract(fast)

// ---------------------------------------------------------------------------
// regrid data movement: prolong new children, restrict new parents
// ---------------------------------------------------------------------------
template <int BI, int BJ, int BK, int NV>
__global__ void __launch_bounds__(NT) k_move(KArgs a, double *Unew, const MoveTask *tasks, int ntasks)
{
    using S = Shape<BI, BJ, BK, NV>;
    for (int it = blockIdx.x; it < ntasks; it += gridDim.x) {
        const MoveTask tk = tasks[it];
        const LevelGeo lg = a.geo[tk.level];
        if (tk.type == MOVE_PROLONG) {
            // one thread per coarse cell of the parent under this child block: 8 fine cells each
            const int ps = tk.src[0];
            const BlockDesc pd = a.desc[ps];
            const LevelGeo cg = a.geo[tk.level - 1];
            constexpr int HI = BI / 2, HJ = BJ / 2, HK = BK / 2;
            for (int c = threadIdx.x; c < HI * HJ * HK; c += blockDim.x) {
                const int h[3] = {c % HI, (c / HI) % HJ, c / (HI * HJ)};
                int g0[3], cl[3], cw[3];
                for (int e = 0; e < 3; ++e) {
                    g0[e] = tk.org[e] + 2 * h[e];
                    cw[e] = g0[e] >> 1;
                    cl[e] = cw[e] - pd.org[e];
                }
                Prolong<NV> P;
                prolong_setup<BI, BJ, BK, NV>(a, ps, cl, cw, cg, lg, g0, P);
                for (int o = 0; o < 8; ++o) {
                    const int li = 2 * h[0] + (o & 1), lj = 2 * h[1] + ((o >> 1) & 1), lk = 2 * h[2] + ((o >> 2) & 1);
                    for (int v = 0; v < NV; ++v) Unew[cidx<S>(tk.dst, v, li, lj, lk)] = P.value(o, v);
                }
            }
            continue;
        }
        for (int c = threadIdx.x; c < S::NC; c += blockDim.x) {
            const int loc[3] = {c % BI, (c / BI) % BJ, c / (BI * BJ)};
            int g[3];
            for (int e = 0; e < 3; ++e) g[e] = tk.org[e] + loc[e];
            {
                const LevelGeo fg = a.geo[tk.level + 1];
                double num[NV], den = 0.0;
                for (int v = 0; v < NV; ++v) num[v] = 0.0;
                for (int o = 0; o < 8; ++o) {
                    const int oo[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
                    int fl[3], oct = 0, fgi[3];
                    for (int e = 0; e < 3; ++e) {
                        const int x = 2 * loc[e] + oo[e];
                        const int q = x / S::dim(e);
                        oct |= q << e;
                        fl[e] = x - q * S::dim(e);
                        fgi[e] = 2 * g[e] + oo[e];
                    }
                    const double wgt = fg.r[fgi[0] + 2].vw * fg.t[fgi[1] + 2].vw * fg.p[fgi[2] + 2].vw;
                    for (int v = 0; v < NV; ++v) num[v] += wgt * a.U[cidx<S>(tk.src[oct], v, fl[0], fl[1], fl[2])];
                    den += wgt;
                }
                for (int v = 0; v < NV; ++v) Unew[cidx<S>(tk.dst, v, loc[0], loc[1], loc[2])] = num[v] / den;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// point sampling (trilinear between cell centres), one work-group per member;
// with t_step set it first ends the step (t += dt, step count + 1, for a
// member with dt > 0), so that the sample carries the new time; the 8 MHD
// primitives are sampled
// ---------------------------------------------------------------------------
template <int BI, int BJ, int BK, int NV>
__global__ void k_sample(KArgs a, const SampleDesc *sd, int nmembers, double *out, double *ring,
                         int *ring_count, int ring_cap, int record, double *t_step, long *nsteps)
{
    using S = Shape<BI, BJ, BK, NV>;
    __shared__ double sw[8][9];                 // per stencil entry: primitives, then its weight
    const int m = blockIdx.x;
    if (m >= nmembers) return;
    if (threadIdx.x == 0 && t_step && a.dt[m] > 0.0) {
        t_step[m] += a.dt[m];
        nsteps[m] += 1;
    }
    if (!sd[m].valid) return;                   // the same for the whole work-group
    const int q = threadIdx.x;                  // entries on 8 threads, loads in flight together
    if (q < 8) {
        const SampleEntry &e = sd[m].e[q];      // read in place (no private copy of the descriptor)
        double u[8];
        if (e.kind == 0) {
            for (int v = 0; v < 8; ++v) u[v] = a.U[cidx<S>(e.slot, v, e.cell[0], e.cell[1], e.cell[2])];
        } else {
            const LevelGeo fg = a.geo[e.level];
            double num[8] = {0, 0, 0, 0, 0, 0, 0, 0}, den = 0.0;
            for (int o = 0; o < 8; ++o) {
                const int oo[3] = {o & 1, (o >> 1) & 1, (o >> 2) & 1};
                const double wgt = fg.r[e.g[0] + oo[0] + 2].vw * fg.t[e.g[1] + oo[1] + 2].vw * fg.p[e.g[2] + oo[2] + 2].vw;
                for (int v = 0; v < 8; ++v)
                    num[v] += wgt * a.U[cidx<S>(e.slot, v, e.cell[0] + oo[0], e.cell[1] + oo[1], e.cell[2] + oo[2])];
                den += wgt;
            }
            for (int v = 0; v < 8; ++v) u[v] = num[v] / den;
        }
        double w[8];
        cons_to_prim(u, w, a.gas);
        for (int v = 0; v < 8; ++v) sw[q][v] = w[v];
        sw[q][8] = e.w;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int e = 0; e < 8; ++e)                 // summed in entry order
        for (int v = 0; v < 8; ++v) acc[v] += sw[e][8] * sw[e][v];
    for (int v = 0; v < 8; ++v) out[m * 8 + v] = acc[v];
    // a launch that ends a step records the sample only for a member that took
    // the step (one past its end time takes dt = 0 and records nothing)
    if (record && !(t_step && !(a.dt[m] > 0.0))) {
        const int c = ring_count[m];
        double *r = ring + ((size_t)m * ring_cap + (c % ring_cap)) * 9;
        r[0] = t_step ? t_step[m] : a.t[m];
        for (int v = 0; v < 8; ++v) r[1 + v] = acc[v];
        ring_count[m] = c + 1;
    }
}

// ---------------------------------------------------------------------------
// instantiations for the supported block shapes
// ---------------------------------------------------------------------------
#define IC_INSTANTIATE_NV(BI, BJ, BK, NV)                                                           \
    template __global__ void k_slabs<BI, BJ, BK, NV, 0>(KArgs, const SlabTask *, const int *);     \
    template __global__ void k_slabs<BI, BJ, BK, NV, 1>(KArgs, const SlabTask *, const int *);     \
    template __global__ void k_reflux<BI, BJ, BK, NV>(KArgs, const RefluxTask *, const int *, const int *); \
    template __global__ void k_rate<BI, BJ, BK, NV>(KArgs);                                        \
    template __global__ void k_divb<BI, BJ, BK, NV>(KArgs);                                        \
    template __global__ void k_clean<BI, BJ, BK, NV>(KArgs);                                       \
    template __global__ void k_indicator<BI, BJ, BK, NV>(KArgs, int8_t *, IndicatorParams);        \
    template __global__ void k_move<BI, BJ, BK, NV>(KArgs, double *, const MoveTask *, int);       \
    template __global__ void k_sample<BI, BJ, BK, NV>(KArgs, const SampleDesc *, int, double *, double *, \
                                                      int *, int, int, double *, long *);
#define IC_INSTANTIATE(BI, BJ, BK) IC_INSTANTIATE_NV(BI, BJ, BK, 8) IC_INSTANTIATE_NV(BI, BJ, BK, 9)

#include "shapes.inc"
#undef IC_INSTANTIATE
#undef IC_INSTANTIATE_NV

// ---------------------------------------------------------------------------
// launchers (kernels are launched from this translation unit)
// ---------------------------------------------------------------------------
namespace {
template <int BI, int BJ, int BK, int NV>
struct L {
    static void slabs(dim3 g, hipStream_t s, const KArgs &a, const SlabTask *t, const int *r, int pass)
    {
        // g: one work-group per task; pass 0 splits a task over SLAB_PARTS,
        // pass 1 gives each task one wave
        if (pass == 0) hipLaunchKernelGGL((k_slabs<BI, BJ, BK, NV, 0>), dim3(g.x * SLAB_PARTS), dim3(NT), 0, s, a, t, r);
        else hipLaunchKernelGGL((k_slabs<BI, BJ, BK, NV, 1>), dim3((g.x + PROLONG_TASKS - 1) / PROLONG_TASKS),
                                dim3(NT), 0, s, a, t, r);
    }
    static void reflux(dim3 g, hipStream_t s, const KArgs &a, const RefluxTask *t, const int *r, const int *n)
    {
        hipLaunchKernelGGL((k_reflux<BI, BJ, BK, NV>), g, dim3(NT), 0, s, a, t, r, n);
    }
    static void rate(dim3 g, hipStream_t s, const KArgs &a)
    {
        hipLaunchKernelGGL((k_rate<BI, BJ, BK, NV>), g, dim3(NT), 0, s, a);
    }
    static void divb(dim3 g, hipStream_t s, const KArgs &a)
    {
        hipLaunchKernelGGL((k_divb<BI, BJ, BK, NV>), g, dim3(NT), 0, s, a);
    }
    static void clean(dim3 g, hipStream_t s, const KArgs &a)
    {
        hipLaunchKernelGGL((k_clean<BI, BJ, BK, NV>), g, dim3(NT), 0, s, a);
    }
    static void indicator(dim3 g, hipStream_t s, const KArgs &a, int8_t *f, const IndicatorParams &p)
    {
        hipLaunchKernelGGL((k_indicator<BI, BJ, BK, NV>), g, dim3(NT), 0, s, a, f, p);
    }
    static void move(dim3 g, hipStream_t s, const KArgs &a, double *Un, const MoveTask *t, int n)
    {
        hipLaunchKernelGGL((k_move<BI, BJ, BK, NV>), g, dim3(NT), 0, s, a, Un, t, n);
    }
    static void sample(dim3 g, hipStream_t s, const KArgs &a, const SampleDesc *sd, int nm, double *out,
                       double *ring, int *cnt, int cap, int rec, double *t_step, long *nsteps)
    {
        hipLaunchKernelGGL((k_sample<BI, BJ, BK, NV>), g, dim3(64), 0, s, a, sd, nm, out, ring, cnt, cap, rec,
                           t_step, nsteps);
    }
    static Launchers get()
    {
        return Launchers{&launch_stage<BI, BJ, BK, NV>, &launch_hancock<BI, BJ, BK, NV>, &divb, &clean, &slabs,
                         &reflux, &rate, &indicator, &move, &sample};
    }
};
}  // namespace

bool get_launchers(int bi, int bj, int bk, int nv, Launchers *out)
{
    if (nv != 8 && nv != 9) return false;
#define IC_INSTANTIATE(BI, BJ, BK)                                                                  \
    if (bi == BI && bj == BJ && bk == BK) {                                                        \
        *out = nv == 8 ? L<BI, BJ, BK, 8>::get() : L<BI, BJ, BK, 9>::get();                         \
        return true;                                                                               \
    }
#include "shapes.inc"
#undef IC_INSTANTIATE
    return false;
}

void launch_dt(hipStream_t s, const KArgs &a, const int *mbeg, const int *mend, int nm, double cfl,
               double dt_fixed, const double *tend, double *dt_last)
{
    hipLaunchKernelGGL(k_dt, dim3(nm), dim3(NT), 0, s, a, mbeg, mend, nm, cfl, dt_fixed, tend, dt_last);
}

void launch_time(hipStream_t s, double *t, const double *dt, long *nsteps, int nm)
{
    hipLaunchKernelGGL(k_time, dim3((nm + 63) / 64), dim3(64), 0, s, t, dt, nsteps, nm);
}
