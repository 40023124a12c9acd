// kernels.hip -- HIP kernels of the Icarus hot path for gfx950 (CDNA4).
//
// k_stage is the fused finite-volume stage (paper Sect. 2.1: TVDLF with a
// Woodward-type limiter, second order): a work-group marches along k (phi)
// through a leaf block (or through 1/2 or 1/4 of it, for short work lists).
// For each k-plane the primitives of the plane and of its two-cell i/j halos
// sit in LDS; every r- and theta-face flux of the plane is computed once by
// one thread and kept in LDS; the phi-face fluxes are computed once per column
// in registers (each of the first 192 or fewer threads owns one (i, j) column
// and carries the previous plane's flux, face state and the next plane's
// primitives).  The update adds the flux differences with the finite-volume
// metric, the hoop, Coriolis, centrifugal and gravity sources, applies the
// floors and writes U_out = U_base + alpha dt L(U).  Meanwhile the last wave,
// which owns no column, copies the next plane's halo and the column plane two
// ahead from HBM into LDS asynchronously.  Halo cells come from neighbouring
// blocks (same level), the block's own edge (outflow) or ghost slabs (inner
// boundary, coarse-fine faces).
#include "kernels.h"

#define NT 256

namespace {

template <class S>
__device__ inline size_t cidx(int slot, int v, int i, int j, int k)
{
    return (size_t)slot * 8 * S::NC + (size_t)v * S::NC + i + S::B0 * (j + S::B1 * k);
}

__device__ inline double wave_max(double x)
{
    for (int off = 32; off > 0; off >>= 1) {
        double y = __shfl_xor(x, off, 64);
        x = x > y ? x : y;
    }
    return x;
}

// Block-wide max over NT threads; result valid in all threads.
__device__ inline double block_max(double x, double *scratch)
{
    x = wave_max(x);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) scratch[wid] = x;
    __syncthreads();
    double m = scratch[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) m = m > scratch[w] ? m : scratch[w];
    __syncthreads();
    return m;
}

}  // namespace

// ---------------------------------------------------------------------------
// fused stage kernel
// ---------------------------------------------------------------------------

// Left and right states at the face between cells c1 and c2 of an LDS line
// c0 c1 c2 c3 (cell stride cs, variable stride vs), reconstructed one
// variable at a time so that only the two face states stay live.  The
// zero-slope fallback of a cell applies when one of its two face densities or
// pressures is not positive.
template <class Rec>
DEV void face_states(const double *p, int cs, int vs, const Rec &r1, const Rec &r2, double L[8], double R[8])
{
    bool ok1 = true, ok2 = true;
#pragma unroll
    for (int v = 0; v < 8; ++v) {
        const double a = p[v * vs], b = p[v * vs + cs], c = p[v * vs + 2 * cs], d = p[v * vs + 3 * cs];
        const double s1 = mc_slope(a, b, c, r1.idm, r1.idp, r1.idc);
        const double s2 = mc_slope(b, c, d, r2.idm, r2.idp, r2.idc);
        L[v] = b + s1 * r1.hp;
        R[v] = c - s2 * r2.hm;
        if (v == 0 || v == 4) {
            ok1 = ok1 && (b - s1 * r1.hm > 0.0) && (L[v] > 0.0);
            ok2 = ok2 && (R[v] > 0.0) && (c + s2 * r2.hp > 0.0);
        }
    }
    if (!ok1) {
#pragma unroll
        for (int v = 0; v < 8; ++v) L[v] = p[v * vs + cs];
    }
    if (!ok2) {
#pragma unroll
        for (int v = 0; v < 8; ++v) R[v] = p[v * vs + 2 * cs];
    }
}

// Cell t of the 4 (BI + BJ) r/theta halo cells of plane k (two layers on each
// side, r-halo first): its (i, j).
template <int BI, int BJ>
DEV void halo_cell(int t, int &i, int &j)
{
    if (t < 4 * BJ) {                 // r-direction halo
        const int side = t / (2 * BJ), rem = t % (2 * BJ);
        const int l = rem / BJ;
        j = rem % BJ;
        i = side ? BI + l : l - 2;
    } else {                          // theta-direction halo
        const int q = t - 4 * BJ;
        const int side = q / (2 * BI), rem = q % (2 * BI);
        const int l = rem / BI;
        i = rem % BI;
        j = side ? BJ + l : l - 2;
    }
}

// Work item of linear work index w when a.xcd_order is set: the work-groups
// of a launch go round-robin to the 8 XCDs (w % 8), so the items are split
// into 8 contiguous runs of the (Morton-ordered) work list, one per XCD, and
// neighbouring blocks -- which read each other's halos -- share an L2.
__device__ inline int xcd_item(int w, int n)
{
    const int q = n >> 3, rem = n & 7;
    const int x = w & 7, pos = w >> 3;
    return x * q + (x < rem ? x : rem) + pos;
}

// W: waves per SIMD the register allocation targets (a tuning choice).
template <int BI, int BJ, int BK, int W>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(W, W)))
k_stage(KArgs a)
{
    using S = Shape<BI, BJ, BK>;
    constexpr int PI = BI + 4, PJ = BJ + 4;
    constexpr int NFI = (BI + 1) * BJ;
    constexpr int NFJ = BI * (BJ + 1);
    constexpr int NCOL = BI * BJ;
    constexpr int NHALO = 4 * (BI + BJ);
    static_assert(NCOL + 64 <= NT && NFI <= 2 * NT && NFJ <= 2 * NT, "plane too large for the work-group");
    // the last wave (it owns no column) copies the next planes asynchronously into LDS
    constexpr int CWAVE = NT / 64 - 1;
    constexpr int NHR = 4 * BJ, NHT = 4 * BI;    // r-halo cells (first), theta-halo cells
    constexpr int NHP = NHR * 8 * 2;             // r-halo: one 4-byte piece per lane, two per double
    constexpr int NTP = NHT / 2 * 8;             // theta-halo rows: one 16-byte piece (two cells) per lane
    constexpr int NCP = NCOL / 2 * 8;            // column plane: one 16-byte piece (two cells) per lane
    static_assert(NCOL % 2 == 0 && BI % 2 == 0 && NCOL <= CWAVE * 64, "column plane copy layout");

    __shared__ double sW[8][PJ][PI];
    __shared__ __attribute__((aligned(16))) double sCol[8][NCOL];     // conserved column plane k+2
    __shared__ __attribute__((aligned(16))) double sHalR[8][NHR];     // conserved r-halo of plane k+1
    __shared__ __attribute__((aligned(16))) double sHalT[8][NHT];     // conserved theta-halo of plane k+1
    // per halo cell: address of variable 0 in plane 0 and the strides (doubles) per variable and plane
    __shared__ const double *sHB[NHALO];
    __shared__ int sHV[NHALO], sHK[NHALO];
    __shared__ double sFi[8][BJ][BI + 1];
    __shared__ double sFj[8][BJ + 1][BI];
    __shared__ RecR sR[BI + 4];
    __shared__ RecT sT[BJ + 4];
    __shared__ double sred[NT / 64];

    const int tid = threadIdx.x;
    const bool col = tid < NCOL;
    const int ci = tid % BI, cj = tid / BI;      // column owned by this thread
    const Gas gs = a.gas;
    const int nitems = *a.nitems;

    const int ks = a.ksplit;                     // parts of the march along k per block
    const int nwork = nitems * ks;
    for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
        const int ww = a.xcd_order ? xcd_item(wi, nwork) : wi;
        const int it = ww / ks, part = ww % ks;
        const int k0 = part * BK / ks, k1 = (part + 1) * BK / ks;
        const int slot = a.items[it];
        struct { int org[3]; int reflux_mask; } bd;
        const int mem = a.desc[slot].member;
        for (int e = 0; e < 3; ++e) bd.org[e] = a.desc[slot].org[e];
        bd.reflux_mask = a.desc[slot].reflux_mask;
        const double dt = a.dt[mem];
        if (dt <= 0.0) continue;                 // member finished: state stays in place
        const LevelGeo lg = a.geo[a.desc[slot].level];
        const double adt = a.alpha * dt;

        __syncthreads();
        for (int m = tid; m < BI + 4; m += NT) sR[m] = lg.r[bd.org[0] + m];
        for (int m = tid; m < BJ + 4; m += NT) sT[m] = lg.t[bd.org[1] + m];

        // --- prologue: column primitives of planes k0 and k0+1, phi-face k0-1/2
        // registers carried along k: Wn = W(k+1), wL = face state of cell k at
        // k+1/2, Fm = flux at k-1/2; W(k) of the own column sits in LDS
        double Wn[8], wL[8], Fm[8];
        int badc = -1;                           // first non-physical input cell of this column
        if (col) {
            double u[8], w0[8], w1[8], lo[8], hi[8], R0[8], Wc[8];
            ghosted8<S>(a, a.U, slot, ci, cj, k0 - 2, u); cons_to_prim(u, w0, gs);
            ghosted8<S>(a, a.U, slot, ci, cj, k0 - 1, u); cons_to_prim(u, w1, gs);
            ghosted8<S>(a, a.U, slot, ci, cj, k0, u);     cons_to_prim(u, Wc, gs);
            ghosted8<S>(a, a.U, slot, ci, cj, k0 + 1, u); cons_to_prim(u, Wn, gs);
            const RecP pm1 = lg.p[bd.org[2] + k0 - 1 + 2], p0 = lg.p[bd.org[2] + k0 + 2];
            reconstruct(w0, w1, Wc, pm1.idm, pm1.idp, pm1.idc, pm1.hm, pm1.hp, lo, hi);
            reconstruct(w1, Wc, Wn, p0.idm, p0.idp, p0.idc, p0.hm, p0.hp, R0, wL);
            rusanov<2>(hi, R0, Fm, gs);
            const int r = k0 == 0 ? a.desc[slot].freg[4] : -1;
            if (r >= 0)
                for (int v = 0; v < 8; ++v) a.freg[(size_t)r * a.reg_stride + ((size_t)v * BJ + cj) * BI + ci] = Fm[v];
#pragma unroll
            for (int v = 0; v < 8; ++v) sW[v][cj + 2][ci + 2] = Wc[v];
        }
        // halos of plane k0, by all threads; the halo address table
        for (int t = tid; t < NHALO; t += NT) {
            int i, j;
            halo_cell<BI, BJ>(t, i, j);
            {
                const double *p0 = ghosted_addr<S>(a.U, a.desc, a.slabs, a.slab_stride, slot, 0, i, j, 0);
                sHB[t] = p0;
                sHV[t] = (int)(ghosted_addr<S>(a.U, a.desc, a.slabs, a.slab_stride, slot, 1, i, j, 0) - p0);
                sHK[t] = (int)(ghosted_addr<S>(a.U, a.desc, a.slabs, a.slab_stride, slot, 0, i, j, 1) - p0);
            }
            double u[8], w[8];
            ghosted8<S>(a, a.U, slot, i, j, k0, u);
            cons_to_prim(u, w, gs);
#pragma unroll
            for (int v = 0; v < 8; ++v) sW[v][j + 2][i + 2] = w[v];
        }
        for (int c = tid; c < NCOL; c += NT) {
            double u[8];
            ghosted8<S>(a, a.U, slot, c % BI, c / BI, k0 + 2, u);
#pragma unroll
            for (int v = 0; v < 8; ++v) sCol[v][c] = u[v];
        }
        double rmax = 0.0;
        __syncthreads();

        for (int k = k0; k < k1; ++k) {
            // plane k with its i/j halos is in LDS

            // (c) r-faces of the plane: face f lies between cells f-1 and f
            for (int t = tid; t < NFI; t += NT) {
                const int f = t % (BI + 1), j = t / (BI + 1);
                double L[8], R[8], fx[8];
                face_states(&sW[0][j + 2][f], 1, PJ * PI, sR[f + 1], sR[f + 2], L, R);
                rusanov<0>(L, R, fx, gs);
#pragma unroll
                for (int v = 0; v < 8; ++v) sFi[v][j][f] = fx[v];
                if (f == 0 || f == BI) {          // raw flux at a coarse-fine face, for the reflux
                    const int r = a.desc[slot].freg[f == 0 ? 0 : 1];
                    if (r >= 0)
                        for (int v = 0; v < 8; ++v) a.freg[(size_t)r * a.reg_stride + ((size_t)v * BK + k) * BJ + j] = fx[v];
                }
            }
            // (d) theta-faces of the plane
            for (int t = tid; t < NFJ; t += NT) {
                const int i = t % BI, f = t / BI;
                double L[8], R[8], fx[8];
                face_states(&sW[0][f][i + 2], PI, PJ * PI, sT[f + 1], sT[f + 2], L, R);
                rusanov<1>(L, R, fx, gs);
#pragma unroll
                for (int v = 0; v < 8; ++v) sFj[v][f][i] = fx[v];
                if (f == 0 || f == BJ) {
                    const int r = a.desc[slot].freg[f == 0 ? 2 : 3];
                    if (r >= 0)
                        for (int v = 0; v < 8; ++v) a.freg[(size_t)r * a.reg_stride + ((size_t)v * BK + k) * BI + i] = fx[v];
                }
            }
            // (e) phi-face k+1/2 of the column: cells k (from LDS), k+1 and k+2
            double Fp[8], Wnext[8];
            if (col) {
                double u[8], W2[8], lo1[8], w0[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) u[v] = sCol[v][tid];
                cons_to_prim(u, W2, gs);
#pragma unroll
                for (int v = 0; v < 8; ++v) w0[v] = sW[v][cj + 2][ci + 2];
                const RecP pk1 = lg.p[bd.org[2] + k + 3];
                double hi1[8];
                reconstruct(w0, Wn, W2, pk1.idm, pk1.idp, pk1.idc, pk1.hm, pk1.hp, lo1, hi1);
                rusanov<2>(wL, lo1, Fp, gs);
                if (k == BK - 1) {
                    const int r = a.desc[slot].freg[5];
                    if (r >= 0)
                        for (int v = 0; v < 8; ++v) a.freg[(size_t)r * a.reg_stride + ((size_t)v * BJ + cj) * BI + ci] = Fp[v];
                }
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    wL[v] = hi1[v];
                    Wnext[v] = Wn[v];
                    Wn[v] = W2[v];
                }
            }
            __syncthreads();

            // (g) update of cell (ci, cj, k)
            if (col) {
                const RecP pk = lg.p[bd.org[2] + k + 2];
                const RecR rr = sR[ci + 2];
                const RecT tt = sT[cj + 2];
                double w[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) w[v] = sW[v][cj + 2][ci + 2];
                if (badc < 0 && unphysical(w)) badc = ci + BI * (cj + BJ * k);
                double acc[8];
                const double thm = rr.rt * tt.thm, thp = rr.rt * tt.thp;
                const double kf = rr.rt * tt.phf * pk.iw;
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    acc[v] = -(rr.ap * sFi[v][cj][ci + 1] - rr.am * sFi[v][cj][ci])
                             - (thp * sFj[v][cj + 1][ci] - thm * sFj[v][cj][ci])
                             - kf * (Fp[v] - Fm[v]);
                }
                if (!a.cart) add_sources(w, rr.rt, tt.ctil, rr.rc, tt.sinc, tt.cosc, a.omega, a.gm, acc);
                const size_t base = cidx<S>(slot, 0, ci, cj, k);
                double unew[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) unew[v] = a.Ubase[base + (size_t)v * S::NC] + adt * acc[v];
                // floors now, or after the reflux for cells on a coarse-fine face
                const int mk = bd.reflux_mask;
                const bool rf = (ci == 0 && (mk & 1)) || (ci == BI - 1 && (mk & 2)) || (cj == 0 && (mk & 4))
                             || (cj == BJ - 1 && (mk & 8)) || (k == 0 && (mk & 16)) || (k == BK - 1 && (mk & 32));
                if (!rf) apply_floors(unew, gs, a.rho_floor, a.p_floor);
#pragma unroll
                for (int v = 0; v < 8; ++v) a.Uout[base + (size_t)v * S::NC] = unew[v];
                if (a.want_rate && !rf) {            // refluxed cells: after the reflux
                    cons_to_prim(unew, w, gs);
                    const double rate = (fabs(w[1]) + fast_speed<0>(w, gs)) * rr.icfl
                                      + (fabs(w[2]) + fast_speed<1>(w, gs)) * rr.irc * tt.icfl
                                      + (fabs(w[3]) + fast_speed<2>(w, gs)) * rr.irc * tt.isinc * pk.iw;
                    rmax = rate > rmax ? rate : rmax;
                }
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    Fm[v] = Fp[v];
                    sW[v][cj + 2][ci + 2] = Wnext[v];   // own cell of plane k+1; read back in (e) and (g)
                }
            } else if (k + 1 < k1 && (tid >> 6) == CWAVE) {
                // (p) meanwhile the last wave (no column) copies the conserved halo of
                // plane k+1 (the update reads no halo cell) and the column plane k+3
                // (read in (e) of the next plane; this plane's copy was read before
                // the last barrier) from HBM into LDS without staging in registers,
                // wait once, and convert the halo to primitives
                const int lane = tid & 63;
                typedef __attribute__((address_space(3))) char lds_t;
#pragma unroll 2
                for (int q = 0; q * 64 < NHP; ++q) {
                    const int g = q * 64 + lane;
                    if (g < NHP) {
                        const int v = g / (2 * NHR), cell = (g >> 1) % NHR, half = g & 1;
                        const char *src = (const char *)(sHB[cell] + v * sHV[cell] + (k + 1) * sHK[cell]) + 4 * half;
                        __builtin_amdgcn_global_load_lds((const void *)src,
                                                         (lds_t *)((lds_t *)&sHalR[0][0] + q * 256), 4, 0, 0);
                    }
                }
#pragma unroll 2
                for (int q = 0; q * 64 < NTP; ++q) {
                    // theta-halo rows are contiguous in i in a block, a slab or an outflow copy
                    const int g = q * 64 + lane;
                    if (g < NTP) {
                        const int v = g / (NHT / 2), cell = NHR + 2 * (g % (NHT / 2));
                        const double *src = sHB[cell] + v * sHV[cell] + (k + 1) * sHK[cell];
                        __builtin_amdgcn_global_load_lds((const void *)src,
                                                         (lds_t *)((lds_t *)&sHalT[0][0] + q * 1024), 16, 0, 0);
                    }
                }
#pragma unroll 2
                for (int q = 0; q * 64 < NCP; ++q) {
                    const int g = q * 64 + lane;
                    if (g < NCP) {
                        const int v = g / (NCOL / 2), pr = g % (NCOL / 2);
                        const double *base = ghosted_addr<S>(a.U, a.desc, a.slabs, a.slab_stride, slot, v, 0, 0, k + 3);
                        __builtin_amdgcn_global_load_lds((const void *)(base + 2 * pr),
                                                         (lds_t *)((lds_t *)&sCol[0][0] + q * 1024), 16, 0, 0);
                    }
                }
                __builtin_amdgcn_s_waitcnt(0);           // this wave's copies have landed
#pragma unroll 1
                for (int t = lane; t < NHALO; t += 64) {
                    int i, j;
                    halo_cell<BI, BJ>(t, i, j);
                    double u[8], w8[8];
#pragma unroll
                    for (int v = 0; v < 8; ++v) u[v] = t < NHR ? sHalR[v][t] : sHalT[v][t - NHR];
                    cons_to_prim(u, w8, gs);
#pragma unroll
                    for (int v = 0; v < 8; ++v) sW[v][j + 2][i + 2] = w8[v];
                }
            }
            __syncthreads();
        }
        if (col && badc >= 0 && atomicCAS(&a.bad[2 * mem], 0, slot + 1) == 0) a.bad[2 * mem + 1] = badc;
        if (a.want_rate) {
            // this part's CFL maximum; the last part clears the unused entries
            const double m = block_max(col ? rmax : 0.0, sred);
            if (tid == 0) a.rate[(size_t)slot * KSPLIT_MAX + part] = m;
            if (part == ks - 1 && tid > part && tid < KSPLIT_MAX) a.rate[(size_t)slot * KSPLIT_MAX + tid] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// Limited linear prolongation from one coarse cell to its 8 children: local
// index cl in the ghosted source block src, wrapped global index cw on level
// geometry cg; the children sit on level geometry lg from the (even,
// unwrapped) global fine index g0 on.  Slopes are minmod of the one-sided
// coordinate differences, applied about the volume centroid of the two
// children along each direction.  A coarse cell whose linear values would
// give any child rho <= 0 or p <= 0 hands its own value to all of them
// (conservative either way).  value(o, v): child o = ox + 2 oy + 4 oz.
struct Prolong {
    double uc[8], sl[3][8], off[3][2];
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

template <int BI, int BJ, int BK>
DEV void prolong_setup(const KArgs &a, int src, const int cl[3], const int cw[3], const LevelGeo &cg,
                       const LevelGeo &lg, const int g0[3], Prolong &P)
{
    using S = Shape<BI, BJ, BK>;
    const double idm[3] = {cg.r[cw[0] + 2].idm, cg.t[cw[1] + 2].idm, cg.p[cw[2] + 2].idm};
    const double idp[3] = {cg.r[cw[0] + 2].idp, cg.t[cw[1] + 2].idp, cg.p[cw[2] + 2].idp};
#pragma unroll
    for (int v = 0; v < 8; ++v) {
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
// One slab task whose face is normal to direction D (a template parameter, so
// that every per-direction index below is a register, not private memory).
// Slab layout: element ((v * 2 + l) * FB + b) * FA + a, layer l = 0 nearest
// the low side.  sP, sOk: LDS for the prolongation's per-parent values.
template <int BI, int BJ, int BK, int D>
DEV void slab_task(const KArgs &a, const SlabTask *tkp, double *sP, int *sOk)
{
    using S = Shape<BI, BJ, BK>;
    constexpr int E1 = tan1(D), E2 = tan2(D);
    constexpr int FA = S::dim(E1), FB = S::dim(E2), Bd = S::dim(D);
    constexpr int NCELL = 2 * FA * FB;
    const int type = tkp->type, side = tkp->face & 1;
    const BlockDesc bd = a.desc[tkp->slot];
    const LevelGeo lg = a.geo[bd.level];
    double *out = a.slabs + (size_t)tkp->slab * a.slab_stride;
    const int g0d = side ? bd.org[D] + Bd : bd.org[D] - 2;     // owner-level index of layer 0 along D
    if (type == SLAB_PROLONG) {
        // children = 2 layers x 2 x 2 fine cells per coarse parent
        constexpr int HA = FA / 2, HB = FB / 2, NP = HA * HB;
        const LevelGeo cg = a.geo[bd.level - 1];
        const int cs = tkp->src[0];
        const int shift[3] = {tkp->shift[0], tkp->shift[1], tkp->shift[2]};
        const int cwrap[3] = {tkp->cwrap[0], tkp->cwrap[1], tkp->cwrap[2]};
        // (1) per parent and variable: coarse value and minmod slopes along r, theta, phi
        for (int t = threadIdx.x; t < NP * 8; t += blockDim.x) {
            const int c = t % NP, v = t / NP;
            int g0[3];
            g0[D] = g0d;
            g0[E1] = bd.org[E1] + 2 * (c % HA);
            g0[E2] = bd.org[E2] + 2 * (c / HA);
            int cl[3], cw[3];
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const int c2 = g0[e] >= 0 ? g0[e] / 2 : -((-g0[e] + 1) / 2);   // floor(g/2)
                cl[e] = c2 + shift[e];
                cw[e] = c2 + cwrap[e];
            }
            const double idm[3] = {cg.r[cw[0] + 2].idm, cg.t[cw[1] + 2].idm, cg.p[cw[2] + 2].idm};
            const double idp[3] = {cg.r[cw[0] + 2].idp, cg.t[cw[1] + 2].idp, cg.p[cw[2] + 2].idp};
            const double uc = ghosted<S>(a.U, a.desc, a.slabs, a.slab_stride, cs, v, cl[0], cl[1], cl[2]);
            double *P = sP + (c * 8 + v) * 4;
            P[0] = uc;
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                int lm[3] = {cl[0], cl[1], cl[2]}, lp[3] = {cl[0], cl[1], cl[2]};
                lm[e] -= 1;
                lp[e] += 1;
                const double um = ghosted<S>(a.U, a.desc, a.slabs, a.slab_stride, cs, v, lm[0], lm[1], lm[2]);
                const double up = ghosted<S>(a.U, a.desc, a.slabs, a.slab_stride, cs, v, lp[0], lp[1], lp[2]);
                const double sa = (uc - um) * idm[e], sb = (up - uc) * idp[e];
                P[1 + e] = sa * sb > 0.0 ? copysign(fmin(fabs(sa), fabs(sb)), sa) : 0.0;
            }
        }
        __syncthreads();
        // (2) per parent: do the linear values give all 8 children rho > 0 and p > 0?
        for (int c = threadIdx.x; c < NP; c += blockDim.x) {
            int g0[3];
            g0[D] = g0d;
            g0[E1] = bd.org[E1] + 2 * (c % HA);
            g0[E2] = bd.org[E2] + 2 * (c / HA);
            const double off[3][2] = {{lg.r[g0[0] + 2].poff, lg.r[g0[0] + 3].poff},
                                      {lg.t[g0[1] + 2].poff, lg.t[g0[1] + 3].poff},
                                      {lg.p[g0[2] + 2].poff, lg.p[g0[2] + 3].poff}};
            const double *P = sP + c * 32;
            bool ok = true;
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                double q[8];
#pragma unroll
                for (int v = 0; v < 8; ++v) {
                    double x = P[v * 4];
                    x += P[v * 4 + 1] * off[0][o & 1];
                    x += P[v * 4 + 2] * off[1][(o >> 1) & 1];
                    x += P[v * 4 + 3] * off[2][(o >> 2) & 1];
                    q[v] = x;
                }
                const double kin = 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0];
                const double mag = 0.5 * (q[5] * q[5] + q[6] * q[6] + q[7] * q[7]);
                ok = ok && q[0] > 0.0 && q[4] - kin - mag > 0.0;
            }
            sOk[c] = ok;
        }
        __syncthreads();
        // (3) the slab element by element (coalesced); a failing parent hands
        // its own value to its children
        for (int e = threadIdx.x; e < 8 * NCELL; e += blockDim.x) {
            const int ia = e % FA, ib = (e / FA) % FB, l = (e / (FA * FB)) & 1, v = e / NCELL;
            const int c = (ia >> 1) + HA * (ib >> 1);
            const double *P = sP + (c * 8 + v) * 4;
            double x = P[0];
            if (sOk[c]) {
                int g[3];
                g[D] = g0d + l;
                g[E1] = bd.org[E1] + ia;
                g[E2] = bd.org[E2] + ib;
                x += P[1] * lg.r[g[0] + 2].poff;
                x += P[2] * lg.t[g[1] + 2].poff;
                x += P[3] * lg.p[g[2] + 2].poff;
            }
            out[e] = x;
        }
        __syncthreads();                            // sP and sOk are reused by the next task
        return;
    }
    const Gas gs = a.gas;
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int ia = c % FA, ib = (c / FA) % FB, l = c / (FA * FB);
        int g[3];                                   // owner-level global index (unwrapped)
        g[D] = g0d + l;
        g[E1] = bd.org[E1] + ia;
        g[E2] = bd.org[E2] + ib;
        double u[8];
        if (type == SLAB_INNER) {
            const int jt = g[1], kp = g[2];
            const int nt = lg.n[1], np = lg.n[2];
            const size_t o = (size_t)jt * np + kp;
            const size_t pl = (size_t)nt * np;
            double w[8];
            w[0] = lg.wind[0 * pl + o];
            w[1] = lg.wind[1 * pl + o];
            w[2] = 0.0;
            w[3] = lg.wind[2 * pl + o];
            w[4] = lg.wind[3 * pl + o];
            w[5] = lg.wind[4 * pl + o];
            w[6] = 0.0;
            w[7] = lg.wind[5 * pl + o];
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
                    }
                }
            }
            prim_to_cons(w, u, gs);
        } else {                                    // SLAB_RESTRICT
            const LevelGeo fg = a.geo[bd.level + 1];
            double num[8] = {0, 0, 0, 0, 0, 0, 0, 0}, den = 0.0;
            int gw[3];
#pragma unroll
            for (int e = 0; e < 3; ++e) gw[e] = g[e] + tkp->shift[e];
            const int fbase[3] = {tkp->fbase[0], tkp->fbase[1], tkp->fbase[2]};
#pragma unroll
            for (int o = 0; o < 8; ++o) {
                int fgi[3], fl[3], q[3];
#pragma unroll
                for (int e = 0; e < 3; ++e) {
                    fgi[e] = 2 * gw[e] + ((o >> e) & 1);
                    const int fb = fgi[e] / S::dim(e);
                    q[e] = fb - fbase[e];
                    fl[e] = fgi[e] - fb * S::dim(e);
                }
                const int fslot = tkp->src[q[E1] + 2 * q[E2]];
                const double wgt = fg.r[fgi[0] + 2].vw * fg.t[fgi[1] + 2].vw * fg.p[fgi[2] + 2].vw;
#pragma unroll
                for (int v = 0; v < 8; ++v) num[v] += wgt * a.U[cidx<S>(fslot, v, fl[0], fl[1], fl[2])];
                den += wgt;
            }
#pragma unroll
            for (int v = 0; v < 8; ++v) u[v] = num[v] / den;
        }
#pragma unroll
        for (int v = 0; v < 8; ++v) out[((size_t)(v * 2 + l) * FB + ib) * FA + ia] = u[v];
    }
}

template <int BI, int BJ, int BK>
__global__ void __launch_bounds__(NT) k_slabs(KArgs a, const SlabTask *tasks, const int *range)
{
    using S = Shape<BI, BJ, BK>;
    __shared__ double sP[S::MAXFACE / 4 * 32];
    __shared__ int sOk[S::MAXFACE / 4];
    const int t0 = range[0], t1 = range[1];
    for (int it = t0 + blockIdx.x; it < t1; it += gridDim.x) {
        const int d = tasks[it].face >> 1;          // uniform over the work-group
        if (d == 0) slab_task<BI, BJ, BK, 0>(a, tasks + it, sP, sOk);
        else if (d == 1) slab_task<BI, BJ, BK, 1>(a, tasks + it, sP, sOk);
        else slab_task<BI, BJ, BK, 2>(a, tasks + it, sP, sOk);
    }
}

// ---------------------------------------------------------------------------
// reflux at coarse-fine faces, then the CFL rates of the corrected cells
// ---------------------------------------------------------------------------
template <int BI, int BJ, int BK>
__device__ inline double cell_rate(const double u[8], const RecR &rr, const RecT &tt, const RecP &pp, const Gas &gs)
{
    double w[8];
    cons_to_prim(u, w, gs);
    return (fabs(w[1]) + fast_speed<0>(w, gs)) * rr.icfl
         + (fabs(w[2]) + fast_speed<1>(w, gs)) * rr.irc * tt.icfl
         + (fabs(w[3]) + fast_speed<2>(w, gs)) * rr.irc * tt.isinc * pp.iw;
}

template <int BI, int BJ, int BK>
__global__ void __launch_bounds__(NT) k_reflux(KArgs a, const RefluxTask *tasks, const int *blocks, const int *nblocks)
{
    using S = Shape<BI, BJ, BK>;
    __shared__ double sred[NT / 64];
    const int nb = *nblocks;
    for (int it = blockIdx.x; it < nb; it += gridDim.x) {
        const int t0 = blocks[2 * it], t1 = blocks[2 * it + 1];
        const int slot = tasks[t0].slot;
        const BlockDesc bd = a.desc[slot];
        const double dt = a.dt[bd.member];
        if (dt <= 0.0) continue;
        const double adt = a.alpha * dt;
        const LevelGeo lg = a.geo[bd.level], fg = a.geo[bd.level + 1];
        for (int q = t0; q < t1; ++q) {
            const RefluxTask tk = tasks[q];
            const int d = tk.face >> 1, side = tk.face & 1;
            const int e1 = tan1(d), e2 = tan2(d);
            const int FA = S::dim(e1), FB = S::dim(e2);
            for (int c = threadIdx.x; c < FA * FB; c += blockDim.x) {
                const int ia = c % FA, ib = c / FA;
                int loc[3];
                loc[d] = side ? S::dim(d) - 1 : 0;
                loc[e1] = ia;
                loc[e2] = ib;
                int g[3];
                for (int e = 0; e < 3; ++e) g[e] = bd.org[e] + loc[e];
                const RecR rr = lg.r[g[0] + 2];
                const RecT tt = lg.t[g[1] + 2];
                const RecP pp = lg.p[g[2] + 2];
                const double Vc = rr.vw * tt.vw * pp.vw;
                double ac;
                if (d == 0) ac = side ? rr.ap : rr.am;
                else if (d == 1) ac = rr.rt * (side ? tt.thp : tt.thm);
                else ac = rr.rt * tt.phf * pp.iw;
                // fine face index along d (global, fine level) and fine tangential cells
                const int gf = 2 * (bd.org[d] + (side ? S::dim(d) : 0));
                double sum[8] = {0, 0, 0, 0, 0, 0, 0, 0};
                for (int ob = 0; ob < 2; ++ob) {
                    for (int oa = 0; oa < 2; ++oa) {
                        const int fa = 2 * ia + oa, fb = 2 * ib + ob;
                        const int qa = fa / FA, qb = fb / FB;
                        const int reg = tk.freg[qa + 2 * qb];
                        int fgl[3];
                        fgl[d] = gf;
                        fgl[e1] = 2 * g[e1] + oa;
                        fgl[e2] = 2 * g[e2] + ob;
                        double A;
                        if (d == 0) A = fg.r[fgl[0] + 2].r2f * fg.t[fgl[1] + 2].vw * fg.p[fgl[2] + 2].vw;
                        else if (d == 1) A = fg.r[fgl[0] + 2].r2h * fg.t[fgl[1] + 2].sf * fg.p[fgl[2] + 2].vw;
                        else A = fg.r[fgl[0] + 2].r2h * fg.t[fgl[1] + 2].dth;
                        const double *F = a.freg + (size_t)reg * a.reg_stride;
                        const int la = fa - qa * FA, lb = fb - qb * FB;
                        for (int v = 0; v < 8; ++v) sum[v] += A * F[((size_t)v * FB + lb) * FA + la];
                    }
                }
                const double *Fc = a.freg + (size_t)tk.creg * a.reg_stride;
                for (int v = 0; v < 8; ++v) {
                    const double corr = ac * Fc[((size_t)v * FB + ib) * FA + ia] - sum[v] / Vc;
                    const size_t o = cidx<S>(slot, v, loc[0], loc[1], loc[2]);
                    a.Uout[o] += side ? adt * corr : -adt * corr;
                }
            }
            __syncthreads();
        }
        // floors on the corrected cells (each once, after all its faces) and
        // their CFL rates; the stage kernel took the maximum over the other cells
        double rmax = 0.0;
        for (int c = threadIdx.x; c < S::NC; c += blockDim.x) {
            const int i = c % BI, j = (c / BI) % BJ, k = c / (BI * BJ);
            const int mk = bd.reflux_mask;
            const bool rf = (i == 0 && (mk & 1)) || (i == BI - 1 && (mk & 2)) || (j == 0 && (mk & 4))
                         || (j == BJ - 1 && (mk & 8)) || (k == 0 && (mk & 16)) || (k == BK - 1 && (mk & 32));
            if (!rf) continue;
            double u[8];
            for (int v = 0; v < 8; ++v) u[v] = a.Uout[cidx<S>(slot, v, i, j, k)];
            apply_floors(u, a.gas, a.rho_floor, a.p_floor);
            for (int v = 0; v < 8; ++v) a.Uout[cidx<S>(slot, v, i, j, k)] = u[v];
            if (a.want_rate) {
                const double r = cell_rate<BI, BJ, BK>(u, lg.r[bd.org[0] + i + 2], lg.t[bd.org[1] + j + 2],
                                                       lg.p[bd.org[2] + k + 2], a.gas);
                rmax = r > rmax ? r : rmax;
            }
        }
        if (a.want_rate) {
            const double m = block_max(rmax, sred);
            if (threadIdx.x == 0) {
                double &r0 = a.rate[(size_t)slot * KSPLIT_MAX];
                r0 = m > r0 ? m : r0;
            }
        }
        __syncthreads();
    }
}

// CFL rate of every leaf (after create, set_state, regrid)
template <int BI, int BJ, int BK>
__global__ void __launch_bounds__(NT) k_rate(KArgs a)
{
    using S = Shape<BI, BJ, BK>;
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
            double u[8], w[8];
            for (int v = 0; v < 8; ++v) u[v] = a.U[cidx<S>(slot, v, i, j, k)];
            cons_to_prim(u, w, a.gas);
            if (bad < 0 && unphysical(w)) bad = c;
            const double r = cell_rate<BI, BJ, BK>(u, lg.r[bd.org[0] + i + 2], lg.t[bd.org[1] + j + 2],
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
        for (int q = mbeg[m] + threadIdx.x; q < mend[m]; q += blockDim.x) {
#pragma unroll
            for (int p = 0; p < KSPLIT_MAX; ++p) {
                const double x = a.rate[(size_t)a.items[q] * KSPLIT_MAX + p];
                r = x > r ? x : r;
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
// ---------------------------------------------------------------------------
#pragma clang fp contract(off)
template <int BI, int BJ, int BK>
__global__ void __launch_bounds__(NT) k_indicator(KArgs a, int8_t *flags, int max_level, double eps,
                                                  double tol_r, double tol_c, double w_rho, double w_v,
                                                  int use_windows, double lon_e, double clt_e,
                                                  double dlon_e, double dclt_e, double dlon_c)
{
    using S = Shape<BI, BJ, BK>;
    const int n = *a.nitems;
    const double PI = 3.14159265358979323846;
    for (int it = blockIdx.x; it < n; it += gridDim.x) {
        const int slot = a.items[it];
        const BlockDesc bd = a.desc[slot];
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
            ghosted8<S>(a, a.U, slot, ijk[0], ijk[1], ijk[2], u);
            cons_to_prim<true>(u, w0, a.gas);
            const double r0 = w0[0];
            const double s0 = sqrt(w0[1] * w0[1] + w0[2] * w0[2] + w0[3] * w0[3]);
            double num_r = 0, den_r = 0, num_v = 0, den_v = 0, dv = 0;
            for (int d = 0; d < 3; ++d) {
                int lo[3] = {ijk[0], ijk[1], ijk[2]}, hi[3] = {ijk[0], ijk[1], ijk[2]};
                lo[d] -= 1;
                hi[d] += 1;
                double wl[8], wh[8];
                ghosted8<S>(a, a.U, slot, lo[0], lo[1], lo[2], u);
                cons_to_prim<true>(u, wl, a.gas);
                ghosted8<S>(a, a.U, slot, hi[0], hi[1], hi[2], u);
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
            if (win && dv < 0.0) {
                if (E > tol_r) hot_r = 1;
                if (E > tol_c) hot_c = 1;
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
template <int BI, int BJ, int BK>
__global__ void __launch_bounds__(NT) k_move(KArgs a, double *Unew, const MoveTask *tasks, int ntasks)
{
    using S = Shape<BI, BJ, BK>;
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
                Prolong P;
                prolong_setup<BI, BJ, BK>(a, ps, cl, cw, cg, lg, g0, P);
                for (int o = 0; o < 8; ++o) {
                    const int li = 2 * h[0] + (o & 1), lj = 2 * h[1] + ((o >> 1) & 1), lk = 2 * h[2] + ((o >> 2) & 1);
                    for (int v = 0; v < 8; ++v) Unew[cidx<S>(tk.dst, v, li, lj, lk)] = P.value(o, v);
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
                double num[8] = {0, 0, 0, 0, 0, 0, 0, 0}, den = 0.0;
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
                    for (int v = 0; v < 8; ++v) num[v] += wgt * a.U[cidx<S>(tk.src[oct], v, fl[0], fl[1], fl[2])];
                    den += wgt;
                }
                for (int v = 0; v < 8; ++v) Unew[cidx<S>(tk.dst, v, loc[0], loc[1], loc[2])] = num[v] / den;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// point sampling (trilinear between cell centres), one work-group per member
// ---------------------------------------------------------------------------
template <int BI, int BJ, int BK>
__global__ void k_sample(KArgs a, const SampleDesc *sd, int nmembers, double *out, double *ring,
                         int *ring_count, int ring_cap, int record)
{
    using S = Shape<BI, BJ, BK>;
    const int m = blockIdx.x;
    if (m >= nmembers || threadIdx.x != 0) return;
    const SampleDesc s = sd[m];
    if (!s.valid) return;
    double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = 0; q < 8; ++q) {
        const SampleEntry e = s.e[q];
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
        for (int v = 0; v < 8; ++v) acc[v] += e.w * w[v];
    }
    for (int v = 0; v < 8; ++v) out[m * 8 + v] = acc[v];
    if (record) {
        const int c = ring_count[m];
        double *r = ring + ((size_t)m * ring_cap + (c % ring_cap)) * 9;
        r[0] = a.t[m];
        for (int v = 0; v < 8; ++v) r[1 + v] = acc[v];
        ring_count[m] = c + 1;
    }
}

// ---------------------------------------------------------------------------
// instantiations for the supported block shapes
// ---------------------------------------------------------------------------
#define IC_INSTANTIATE(BI, BJ, BK)                                                                  \
    template __global__ void k_stage<BI, BJ, BK, 1>(KArgs);                                        \
    template __global__ void k_stage<BI, BJ, BK, 2>(KArgs);                                        \
    template __global__ void k_slabs<BI, BJ, BK>(KArgs, const SlabTask *, const int *);            \
    template __global__ void k_reflux<BI, BJ, BK>(KArgs, const RefluxTask *, const int *, const int *); \
    template __global__ void k_rate<BI, BJ, BK>(KArgs);                                            \
    template __global__ void k_indicator<BI, BJ, BK>(KArgs, int8_t *, int, double, double, double, \
                                                     double, double, int, double, double, double,  \
                                                     double, double);                              \
    template __global__ void k_move<BI, BJ, BK>(KArgs, double *, const MoveTask *, int);           \
    template __global__ void k_sample<BI, BJ, BK>(KArgs, const SampleDesc *, int, double *, double *, \
                                                  int *, int, int);

#include "shapes.inc"
#undef IC_INSTANTIATE

// ---------------------------------------------------------------------------
// launchers (kernels are launched from this translation unit)
// ---------------------------------------------------------------------------
namespace {
template <int BI, int BJ, int BK>
struct L {
    static void stage(dim3 g, hipStream_t s, const KArgs &a, int waves)
    {
        if (waves == 1) hipLaunchKernelGGL((k_stage<BI, BJ, BK, 1>), g, dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((k_stage<BI, BJ, BK, 2>), g, dim3(NT), 0, s, a);
    }
    static void slabs(dim3 g, hipStream_t s, const KArgs &a, const SlabTask *t, const int *r)
    {
        hipLaunchKernelGGL((k_slabs<BI, BJ, BK>), g, dim3(NT), 0, s, a, t, r);
    }
    static void reflux(dim3 g, hipStream_t s, const KArgs &a, const RefluxTask *t, const int *b, const int *n)
    {
        hipLaunchKernelGGL((k_reflux<BI, BJ, BK>), g, dim3(NT), 0, s, a, t, b, n);
    }
    static void rate(dim3 g, hipStream_t s, const KArgs &a) { hipLaunchKernelGGL((k_rate<BI, BJ, BK>), g, dim3(NT), 0, s, a); }
    static void indicator(dim3 g, hipStream_t s, const KArgs &a, int8_t *f, const IndicatorParams &p)
    {
        hipLaunchKernelGGL((k_indicator<BI, BJ, BK>), g, dim3(NT), 0, s, a, f, p.max_level, p.eps, p.tol_r,
                           p.tol_c, p.w_rho, p.w_v, p.use_windows, p.lon_e, p.clt_e, p.dlon_e, p.dclt_e,
                           p.dlon_c);
    }
    static void move(dim3 g, hipStream_t s, const KArgs &a, double *Un, const MoveTask *t, int n)
    {
        hipLaunchKernelGGL((k_move<BI, BJ, BK>), g, dim3(NT), 0, s, a, Un, t, n);
    }
    static void sample(dim3 g, hipStream_t s, const KArgs &a, const SampleDesc *sd, int nm, double *out,
                       double *ring, int *cnt, int cap, int rec)
    {
        hipLaunchKernelGGL((k_sample<BI, BJ, BK>), g, dim3(64), 0, s, a, sd, nm, out, ring, cnt, cap, rec);
    }
};
}  // namespace

bool get_launchers(int bi, int bj, int bk, Launchers *out)
{
#define IC_INSTANTIATE(BI, BJ, BK)                                                                  \
    if (bi == BI && bj == BJ && bk == BK) {                                                        \
        *out = Launchers{&L<BI, BJ, BK>::stage, &L<BI, BJ, BK>::slabs, &L<BI, BJ, BK>::reflux,     \
                         &L<BI, BJ, BK>::rate, &L<BI, BJ, BK>::indicator, &L<BI, BJ, BK>::move,    \
                         &L<BI, BJ, BK>::sample};                                                  \
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
