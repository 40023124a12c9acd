// stage.hip -- the fused finite-volume stage kernel of the Icarus hot path (gfx950, CDNA4).
//
// k_stage is the fused finite-volume stage (paper Sect. 2.1: TVDLF with a
// Woodward-type limiter, second order): a work-group marches along k (phi)
// through a leaf block (or through a part of it, down to one plane, for short
// work lists).
// For each k-plane the primitives of the plane and of its two-cell i/j halos
// sit in LDS; every cell is reconstructed once per direction, and every r- and
// theta-face flux of the plane is computed once by one thread (which takes the
// left state from its neighbouring lane through LDS) and kept in LDS; the
// phi-face fluxes are computed once per column
// in registers (each of the first 192 or fewer threads owns one (i, j) column
// and carries the previous plane's flux, face state and the next plane's
// primitives).  The update adds the flux differences with the finite-volume
// metric, the hoop, Coriolis, centrifugal and gravity sources, applies the
// floors and writes U_out = U_base + alpha dt L(U).  The last wave, which owns
// no column, starts the asynchronous HBM-to-LDS copy of the next plane's halo
// once its share of the plane's r/theta fluxes is done; during the update it
// starts the copy of the column plane three ahead, waits for both and converts
// the halo to primitives.  Halo cells come from neighbouring blocks (same
// level), the block's own edge (outflow) or ghost slabs (inner boundary,
// coarse-fine faces).  The block's phi metric records sit in LDS.
#include "common.h"

// ---------------------------------------------------------------------------
// fused stage kernel
// ---------------------------------------------------------------------------

// Cell t of the 4 (BI + BJ) r/theta halo cells of plane k (two layers on each
// side, r-halo first, its two layers of one j adjacent): its (i, j).
template <int BI, int BJ>
DEV void halo_cell(int t, int &i, int &j)
{
    if (t < 4 * BJ) {                 // r-direction halo
        const int side = t / (2 * BJ), rem = t % (2 * BJ);
        const int l = rem % 2;
        j = rem / 2;
        i = side ? BI + l : l - 2;
    } else {                          // theta-direction halo
        const int q = t - 4 * BJ;
        const int side = q / (2 * BI), rem = q % (2 * BI);
        const int l = rem / BI;
        i = rem % BI;
        j = side ? BJ + l : l - 2;
    }
}

// Conserved state of the column (ci, cj) in k-plane k (possibly a ghost plane).
template <class S>
DEV void column_u(const KArgs &a, int slot, const Faces &nb, int ci, int cj, int k, double *u)
{
    const int off = ci + S::B0 * cj;
#pragma unroll
    for (int v = 0; v < S::NV; ++v) u[v] = cell_addr<S>(a.U, a.slabs, a.slab_stride, slot, nb, v, 0, 0, k)[off];
}

// Halo cells of one r- or theta-face of a block (d = 0 or 1): the cell of
// layer l (0 nearest the low side), in-face index a (j on an r-face, i on a
// theta-face), plane k and variable v is at base + l sl + a sa + k sk + v sv
// in the same-level neighbour, the block's own edge (outflow) or the ghost
// slab -- the cases of cell_addr, resolved once per face.
struct FaceMap {
    const double *base;
    int sl, sa, sk, sv;
};

template <class S>
DEV FaceMap face_map(const KArgs &a, int slot, const Faces &nb, int d, int side)
{
    const int Bd = S::dim(d);
    const int code = face_code(nb, 2 * d + side);
    FaceMap m;
    if (code >= 0 || code == NBR_OUTFLOW) {
        const int blk = code >= 0 ? code : slot;
        const int i0 = code >= 0 ? (side ? 0 : Bd - 2) : (side ? Bd - 1 : 0);   // layer 0 along d
        const int sl = code >= 0 ? 1 : 0;
        m.base = a.U + (size_t)blk * S::NV * S::NC + (d == 0 ? i0 : S::B0 * i0);
        m.sl = d == 0 ? sl : S::B0 * sl;
        m.sa = d == 0 ? S::B0 : 1;
        m.sk = S::B0 * S::B1;
        m.sv = S::NC;
    } else {
        const int FA = d == 0 ? S::B1 : S::B0, FB = S::B2;    // slab layout of cell_addr
        m.base = a.slabs + (size_t)nbr_slab(code) * a.slab_stride;
        m.sl = FB * FA;
        m.sa = 1;
        m.sk = FA;
        m.sv = 2 * FB * FA;
    }
    return m;
}

// A radial metric record in LDS, padded from 16 to 17 doubles: the lanes of a
// row read the records of consecutive cells, and at a 16-double stride every
// second record falls on the same LDS banks (a 9-way conflict on each field
// for a row of 18 lanes); at 17 the 32 lanes of a half-wave meet 32 distinct
// bank pairs.
struct RecRPad {
    RecR r;
    double pad;
};

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

// NV: conserved variables (8, or 9 with the tracer); W: waves per SIMD the
// register allocation targets (a tuning choice); LIM: the limiter of the
// reconstruction (LIM_MC, the paper's, by default).
template <int BI, int BJ, int BK, int NV, int W, int LIM>
__global__ void __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(W, W)))
k_stage(KArgs a)
{
    using S = Shape<BI, BJ, BK, NV>;
    constexpr int PI = BI + 4, PJ = BJ + 4;
    constexpr int NFI = (BI + 1) * BJ;
    constexpr int NFJ = BI * (BJ + 1);
    constexpr int NCOL = BI * BJ;
    constexpr int NHALO = 4 * (BI + BJ);
    static_assert(NCOL + 64 <= NT && NFI <= 2 * NT && NFJ <= 2 * NT, "plane too large for the work-group");
    // the last wave (it owns no column) copies the next planes asynchronously into LDS
    constexpr int CWAVE = NT / 64 - 1;
    constexpr int NHR = 4 * BJ, NHT = 4 * BI;    // r-halo cells (first), theta-halo cells
    constexpr int NHP = NHR * NV * 2;            // r-halo: one 4-byte piece per lane, two per double
    constexpr int NHQ = NHR / 2 * NV;            // r-halo between same-level blocks: one 16-byte piece (two layers) per lane
    constexpr int NTP = NHT / 2 * NV;            // theta-halo rows: one 16-byte piece (two cells) per lane
    constexpr int NCP = NCOL / 2 * NV;           // column plane: one 16-byte piece (two cells) per lane
    static_assert(NCOL % 2 == 0 && BI % 2 == 0 && NCOL <= CWAVE * 64, "column plane copy layout");

    __shared__ double sW[NV][PJ][PI];
    __shared__ __attribute__((aligned(16))) double sCol[NV][NCOL];     // conserved column plane k+2
    __shared__ __attribute__((aligned(16))) double sHalR[NV][NHR];     // conserved r-halo of plane k+1
    __shared__ __attribute__((aligned(16))) double sHalT[NV][NHT];     // conserved theta-halo of plane k+1
    // per halo cell: address of variable 0 in plane 0 and the strides (doubles) per variable and plane
    __shared__ const double *sHB[NHALO];
    __shared__ int sHV[NHALO], sHK[NHALO];
    __shared__ double sFi[NV][BJ][BI + 1];
    // theta fluxes; rows padded so that the lanes of (d), which walk the rows,
    // spread over the LDS banks (a row of 16 doubles would map every second row
    // onto the same banks)
    constexpr int SJ = BI % 8 == 0 ? BI + 4 : BI;
    __shared__ double sFj[NV][BJ + 1][SJ];
    __shared__ RecRPad sR[BI + 4];
    __shared__ RecT sT[BJ + 4];
    __shared__ RecP sP[BK + 4];
    __shared__ double sred[NT / 64];

    const Gas gs = a.gas;
    const int nitems = *a.nitems;

    const int ks = a.ksplit;                     // parts of the march along k per block
    const int nwork = nitems * ks;
    for (int wi = blockIdx.x; wi < nwork; wi += gridDim.x) {
        // the thread index, opaque to the compiler once per work item: the
        // addresses and masks derived from it are formed per item instead of
        // being kept live (or spilled) across the whole kernel
        int tid = threadIdx.x;
        asm volatile("" : "+v"(tid));
        const bool col = tid < NCOL;
        const int ci = tid % BI, cj = tid / BI;      // column owned by this thread
        const int ww = a.xcd_order ? xcd_item(wi, nwork) : wi;
        const int it = ww / ks, part = ww % ks;
        const int k0 = part * BK / ks, k1 = (part + 1) * BK / ks;
        const int slot = a.items[it];
        // block descriptor in scalar registers (only constant indices into bd)
        struct { int org[3]; int reflux_mask; int freg[6]; } bd;
        const int mem = a.desc[slot].member;
        for (int e = 0; e < 3; ++e) bd.org[e] = a.desc[slot].org[e];
        bd.reflux_mask = a.desc[slot].reflux_mask;
        // both r-neighbours on the same level: the two halo layers of a row are
        // adjacent cells of the neighbour (else an outflow copy or a ghost slab)
        const bool rpair = a.desc[slot].nbr[0] >= 0 && a.desc[slot].nbr[1] >= 0;
        for (int e = 0; e < 6; ++e) bd.freg[e] = a.desc[slot].freg[e];
        const Faces nb = load_faces(a.desc, slot);
        const double dt = a.dt[mem];
        if (dt <= 0.0) continue;                 // member finished: state stays in place
        const LevelGeo lg = a.geo[a.desc[slot].level];
        const double adt = a.alpha * dt;

        __syncthreads();
        for (int m = tid; m < BI + 4; m += NT) sR[m].r = lg.r[bd.org[0] + m];
        for (int m = tid; m < BJ + 4; m += NT) sT[m] = lg.t[bd.org[1] + m];
        for (int m = tid; m < BK + 4; m += NT) sP[m] = lg.p[bd.org[2] + m];
        // (the metric tables are read after the barrier that ends the prologue)

        // --- prologue: column primitives of planes k0 and k0+1, phi-face k0-1/2
        // registers carried along k: Wn = W(k+1), wL = face state of cell k at
        // k+1/2, Fm = flux at k-1/2; W(k) of the own column sits in LDS
        double Wn[NV], wL[NV], Fm[NV];
        int badc = -1;                           // first non-physical input (or stage-2 output) cell of this column
        int nfr = 0, nfp = 0;                    // cells of this column the density / pressure floor acted on
        if (col) {
            double u[NV], w0[NV], w1[NV], lo[NV], hi[NV], R0[NV], Wc[NV];
            column_u<S>(a, slot, nb, ci, cj, k0 - 2, u); cons_to_prim<false, NV>(u, w0, gs);
            column_u<S>(a, slot, nb, ci, cj, k0 - 1, u); cons_to_prim<false, NV>(u, w1, gs);
            column_u<S>(a, slot, nb, ci, cj, k0, u);     cons_to_prim<false, NV>(u, Wc, gs);
            column_u<S>(a, slot, nb, ci, cj, k0 + 1, u); cons_to_prim<false, NV>(u, Wn, gs);
            const RecP pm1 = lg.p[bd.org[2] + k0 + 1], p0 = lg.p[bd.org[2] + k0 + 2];
            reconstruct<LIM, NV>(w0, w1, Wc, pm1.idm, pm1.idp, pm1.idc, pm1.hm, pm1.hp, lo, hi);
            reconstruct<LIM, NV>(w1, Wc, Wn, p0.idm, p0.idp, p0.idc, p0.hm, p0.hp, R0, wL);
            rusanov<2, NV>(hi, R0, Fm, gs);
            const int r = k0 == 0 ? bd.freg[4] : -1;
            if (r >= 0)
                for (int v = 0; v < NV; ++v) a.freg[(size_t)r * a.reg_stride + ((size_t)v * BJ + cj) * BI + ci] = Fm[v];
#pragma unroll
            for (int v = 0; v < NV; ++v) sW[v][cj + 2][ci + 2] = Wc[v];
        }
        // halos of plane k0 and the halo address table (a halo cell's address
        // is affine in v and in k within the block's k-range), by the threads
        // that own no column beside the column prologue, one cell each; where
        // the halo has more cells than they are threads, the last column
        // threads take one cell each as well (their loads go out with the
        // column loads; all loads first)
        {
            constexpr int NSP = NT - NCOL;
            constexpr int NXH = NHALO > NSP ? NHALO - NSP : 0;
            static_assert(NXH <= 64 && NHALO <= NSP + NXH, "halo cells per thread");
            constexpr int HIT = NXH > 0 ? 1 : (NHALO + NSP - 1) / NSP;
            const bool helper = NXH > 0 && col && tid >= NCOL - NXH;
            const int tb = col ? (helper ? NSP + tid - (NCOL - NXH) : NHALO) : tid - NCOL;
            if (tb < NHALO) {
                const FaceMap fm[4] = {face_map<S>(a, slot, nb, 0, 0), face_map<S>(a, slot, nb, 0, 1),
                                       face_map<S>(a, slot, nb, 1, 0), face_map<S>(a, slot, nb, 1, 1)};
                double u[HIT][NV];
#pragma unroll
                for (int h = 0; h < HIT; ++h) {
                    const int t = tb + h * NSP;
                    if (t < NHALO) {
                        int i, j;
                        halo_cell<BI, BJ>(t, i, j);
                        const bool rh = t < NHR;                  // r-halo, else theta-halo
                        const int idx = rh ? i : j, bd_ = rh ? BI : BJ;
                        const int side = idx >= bd_ ? 1 : 0, l = side ? idx - bd_ : idx + 2, q = rh ? j : i;
                        const int f = (rh ? 0 : 2) + side;
                        const FaceMap &m0 = fm[0], &m1 = fm[1], &m2 = fm[2], &m3 = fm[3];
                        const double *fb = f == 0 ? m0.base : f == 1 ? m1.base : f == 2 ? m2.base : m3.base;
                        const int fl = f == 0 ? m0.sl : f == 1 ? m1.sl : f == 2 ? m2.sl : m3.sl;
                        const int fa = f == 0 ? m0.sa : f == 1 ? m1.sa : f == 2 ? m2.sa : m3.sa;
                        const int hk = f == 0 ? m0.sk : f == 1 ? m1.sk : f == 2 ? m2.sk : m3.sk;
                        const int hv = f == 0 ? m0.sv : f == 1 ? m1.sv : f == 2 ? m2.sv : m3.sv;
                        const double *p0 = fb + l * fl + q * fa;
                        sHB[t] = p0;
                        sHV[t] = hv;
                        sHK[t] = hk;
#pragma unroll
                        for (int v = 0; v < NV; ++v) u[h][v] = p0[v * hv + k0 * hk];
                    }
                }
#pragma unroll
                for (int h = 0; h < HIT; ++h) {
                    const int t = tb + h * NSP;
                    if (t < NHALO) {
                        int i, j;
                        halo_cell<BI, BJ>(t, i, j);
                        double w[NV];
                        cons_to_prim<false, NV>(u[h], w, gs);
#pragma unroll
                        for (int v = 0; v < NV; ++v) sW[v][j + 2][i + 2] = w[v];
                    }
                }
            }
        }
        for (int c = tid; c < NCOL; c += NT) {
            double u[NV];
            column_u<S>(a, slot, nb, c % BI, c / BI, k0 + 2, u);
#pragma unroll
            for (int v = 0; v < NV; ++v) sCol[v][c] = u[v];
        }
        double rmax = 0.0;
        __syncthreads();

        for (int k = k0; k < k1; ++k) {
            // plane k with its i/j halos is in LDS
            // (c) r-faces of the plane.  A row of lanes takes the cells c = -1 .. BI
            // of one j: each lane reconstructs its cell's two face states once,
            // passes the upper one to the next lane through LDS (a row lies within
            // one wave, whose LDS accesses stay in order) and computes the flux at
            // its lower face f = c, between cells c-1 and c.
            {
                constexpr int RL = BI + 2, RPW = 64 / RL;
                static_assert((BJ + RPW - 1) / RPW <= NT / 64, "r-face rows per wave");
                const int lane = tid & 63, c = lane % RL - 1;
                const int j = (tid >> 6) * RPW + lane / RL;
                const bool act = lane < RPW * RL && j < BJ;
                double lo[NV], hi[NV];
                if (act) {
                    double wm[NV], w0[NV], wp[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        wm[v] = sW[v][j + 2][c + 1];
                        w0[v] = sW[v][j + 2][c + 2];
                        wp[v] = sW[v][j + 2][c + 3];
                    }
                    const RecR rc = sR[c + 2].r;
                    reconstruct<LIM, NV>(wm, w0, wp, rc.idm, rc.idp, rc.idc, rc.hm, rc.hp, lo, hi);
                    if (c < BI)
#pragma unroll
                        for (int v = 0; v < NV; ++v) sFi[v][j][c + 1] = hi[v];
                }
                __builtin_amdgcn_wave_barrier();
                if (act && c >= 0) {
                    double L[NV], fx[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) L[v] = sFi[v][j][c];
                    rusanov<0, NV>(L, lo, fx, gs);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sFi[v][j][c] = fx[v];
                    if (c == 0 || c == BI) {      // raw flux at a coarse-fine face, for the reflux
                        const int r = c == 0 ? bd.freg[0] : bd.freg[1];
                        if (r >= 0)
                            for (int v = 0; v < NV; ++v)
                                a.freg[(size_t)r * a.reg_stride + ((size_t)v * BK + k) * BJ + j] = fx[v];
                    }
                }
            }
            // (d) theta-faces of the plane, the same way along j: a column of lanes
            // takes the cells c = -1 .. BJ of one i (the columns of a wave interleaved)
            {
                constexpr int CL = BJ + 2, CPW = 64 / CL;
                static_assert((BI + CPW - 1) / CPW <= NT / 64, "theta-face columns per wave");
                const int lane = tid & 63, c = lane / CPW - 1;
                const int i = (tid >> 6) * CPW + lane % CPW;
                const bool act = lane < CPW * CL && i < BI;
                double lo[NV], hi[NV];
                if (act) {
                    double wm[NV], w0[NV], wp[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        wm[v] = sW[v][c + 1][i + 2];
                        w0[v] = sW[v][c + 2][i + 2];
                        wp[v] = sW[v][c + 3][i + 2];
                    }
                    const RecT rc = sT[c + 2];
                    reconstruct<LIM, NV>(wm, w0, wp, rc.idm, rc.idp, rc.idc, rc.hm, rc.hp, lo, hi);
                    if (c < BJ)
#pragma unroll
                        for (int v = 0; v < NV; ++v) sFj[v][c + 1][i] = hi[v];
                }
                __builtin_amdgcn_wave_barrier();
                if (act && c >= 0) {
                    double L[NV], fx[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) L[v] = sFj[v][c][i];
                    rusanov<1, NV>(L, lo, fx, gs);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sFj[v][c][i] = fx[v];
                    if (c == 0 || c == BJ) {
                        const int r = c == 0 ? bd.freg[2] : bd.freg[3];
                        if (r >= 0)
                            for (int v = 0; v < NV; ++v)
                                a.freg[(size_t)r * a.reg_stride + ((size_t)v * BK + k) * BI + i] = fx[v];
                    }
                }
            }
            if (k + 1 < k1 && (tid >> 6) == CWAVE) {
                // the last wave, done with its LDS work of this phase, starts the
                // copies of the conserved r/theta halo of plane k+1 into LDS (read
                // before the last barrier); they land while the other waves finish
                // the plane's fluxes (a wave's LDS accesses wait for its own copies
                // into LDS, so it issues them after its own reads)
                const int lane = tid & 63;
                typedef __attribute__((address_space(3))) char lds_t;
                if (rpair) {
#pragma unroll 2
                    for (int q = 0; q * 64 < NHQ; ++q) {
                        const int g = q * 64 + lane;
                        if (g < NHQ) {
                            const int v = g / (NHR / 2), cell = 2 * (g % (NHR / 2));
                            const double *src = sHB[cell] + v * sHV[cell] + (k + 1) * sHK[cell];
                            __builtin_amdgcn_global_load_lds((const void *)src,
                                                             (lds_t *)((lds_t *)&sHalR[0][0] + q * 1024), 16, 0, 0);
                        }
                    }
                } else {
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
            }

            // (e) phi-face k+1/2 of the column: cells k (from LDS), k+1 and k+2
            double Fp[NV], Wnext[NV];
            if (col) {
                double u[NV], W2[NV], lo1[NV], w0[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) u[v] = sCol[v][tid];
                cons_to_prim<false, NV>(u, W2, gs);
#pragma unroll
                for (int v = 0; v < NV; ++v) w0[v] = sW[v][cj + 2][ci + 2];
                const RecP pk1 = sP[k + 3];
                double hi1[NV];
                reconstruct<LIM, NV>(w0, Wn, W2, pk1.idm, pk1.idp, pk1.idc, pk1.hm, pk1.hp, lo1, hi1);
                rusanov<2, NV>(wL, lo1, Fp, gs);
                if (k == BK - 1) {
                    const int r = bd.freg[5];
                    if (r >= 0)
                        for (int v = 0; v < NV; ++v) a.freg[(size_t)r * a.reg_stride + ((size_t)v * BJ + cj) * BI + ci] = Fp[v];
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    wL[v] = hi1[v];
                    Wnext[v] = Wn[v];
                    Wn[v] = W2[v];
                }
            }
            __syncthreads();

            // (g) update of cell (ci, cj, k)
            if (col) {
                const RecP pk = sP[k + 2];
                const RecR rr = sR[ci + 2].r;
                const RecT tt = sT[cj + 2];
                double w[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) w[v] = sW[v][cj + 2][ci + 2];
                if (badc < 0 && unphysical<NV>(w)) badc = ci + BI * (cj + BJ * k);
                double acc[NV];
                const double thm = rr.rt * tt.thm, thp = rr.rt * tt.thp;
                const double kf = rr.rt * tt.phf * pk.iw;
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    acc[v] = -(rr.ap * sFi[v][cj][ci + 1] - rr.am * sFi[v][cj][ci])
                             - (thp * sFj[v][cj + 1][ci] - thm * sFj[v][cj][ci])
                             - kf * (Fp[v] - Fm[v]);
                }
                if (!a.cart) add_sources(w, rr.rt, tt.ctil, rr.rc, tt.sinc, tt.cosc, a.omega, a.gm, acc);
                const size_t base = cidx<S>(slot, 0, ci, cj, k);
                double unew[NV];
#pragma unroll
                for (int v = 0; v < NV; ++v) unew[v] = a.Ubase[base + (size_t)v * S::NC] + adt * acc[v];
                // floors now, or after the reflux for cells on a coarse-fine face
                const int mk = bd.reflux_mask;
                const bool rf = (ci == 0 && (mk & 1)) || (ci == BI - 1 && (mk & 2)) || (cj == 0 && (mk & 4))
                             || (cj == BJ - 1 && (mk & 8)) || (k == 0 && (mk & 16)) || (k == BK - 1 && (mk & 32));
                if (!rf) {
                    const int f = apply_floors(unew, gs, a.rho_floor, a.p_floor);
                    nfr += f & 1;
                    nfp += f >> 1;
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) a.Uout[base + (size_t)v * S::NC] = unew[v];
                if (a.want_rate && !rf) {            // refluxed cells: after the reflux
                    cons_to_prim<false, NV>(unew, w, gs);
                    // the step's result: a non-finite value created in this stage
                    // would otherwise drop out of the CFL maximum unnoticed
                    if (badc < 0 && unphysical<NV>(w)) badc = ci + BI * (cj + BJ * k);
                    const double rate = (fabs(w[1]) + fast_speed<0>(w, gs)) * rr.icfl
                                      + (fabs(w[2]) + fast_speed<1>(w, gs)) * rr.irc * tt.icfl
                                      + (fabs(w[3]) + fast_speed<2>(w, gs)) * rr.irc * tt.isinc * pk.iw;
                    rmax = rate > rmax ? rate : rmax;
                }
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    Fm[v] = Fp[v];
                    sW[v][cj + 2][ci + 2] = Wnext[v];   // own cell of plane k+1; read back in (e) and (g)
                }
            } else if (k + 1 < k1 && (tid >> 6) == CWAVE) {
                // (p) meanwhile the last wave (no column) starts the copy of the
                // column plane k+3 from HBM into LDS (read in (e) of the next plane;
                // this plane's copy was read before the last barrier), waits for it
                // and for the halo copies of plane k+1, and converts that halo to
                // primitives
                const int lane = tid & 63;
                typedef __attribute__((address_space(3))) char lds_t;
#pragma unroll 2
                for (int q = 0; q * 64 < NCP; ++q) {
                    const int g = q * 64 + lane;
                    if (g < NCP) {
                        const int v = g / (NCOL / 2), pr = g % (NCOL / 2);
                        const double *base = cell_addr<S>(a.U, a.slabs, a.slab_stride, slot, nb, v, 0, 0, k + 3);
                        __builtin_amdgcn_global_load_lds((const void *)(base + 2 * pr),
                                                         (lds_t *)((lds_t *)&sCol[0][0] + q * 1024), 16, 0, 0);
                    }
                }
                __builtin_amdgcn_s_waitcnt(0);           // column plane k+3 and the halo have landed
#pragma unroll 1
                for (int t = lane; t < NHALO; t += 64) {
                    int i, j;
                    halo_cell<BI, BJ>(t, i, j);
                    double u[NV], w8[NV];
#pragma unroll
                    for (int v = 0; v < NV; ++v) u[v] = t < NHR ? sHalR[v][t] : sHalT[v][t - NHR];
                    cons_to_prim<false, NV>(u, w8, gs);
#pragma unroll
                    for (int v = 0; v < NV; ++v) sW[v][j + 2][i + 2] = w8[v];
                }
            }
            __syncthreads();
        }
        if (col && badc >= 0 && atomicCAS(&a.bad[2 * mem], 0, slot + 1) == 0) a.bad[2 * mem + 1] = badc;
        if (col && (nfr | nfp)) {
            atomicAdd(&a.floors[2 * mem], (unsigned long long)nfr);
            atomicAdd(&a.floors[2 * mem + 1], (unsigned long long)nfp);
        }
        if (a.want_rate) {
            // this part's CFL maximum; the last part clears the unused entries
            const double m = block_max(col ? rmax : 0.0, sred);
            if (tid == 0) a.rate[(size_t)slot * KSPLIT_MAX + part] = m;
            if (part == ks - 1 && tid > part && tid < KSPLIT_MAX) a.rate[(size_t)slot * KSPLIT_MAX + tid] = 0.0;
        }
    }
}

// ---------------------------------------------------------------------------
// instantiations and launch
// ---------------------------------------------------------------------------
// the other limiters are built for two waves per SIMD only; the tracer (NV =
// 9) with two waves per SIMD where two work-groups' LDS fits a CU (one on
// planes of more than 160 cells), every limiter
template <int BI, int BJ, int BK, int NV>
void launch_stage(dim3 g, hipStream_t s, const KArgs &a, int waves, int limiter)
{
    if constexpr (NV > 8) {
        constexpr int W9 = BI * BJ > 160 ? 1 : 2;
        if (limiter == LIM_MINMOD) hipLaunchKernelGGL((k_stage<BI, BJ, BK, NV, W9, LIM_MINMOD>), g, dim3(NT), 0, s, a);
        else if (limiter == LIM_VANLEER)
            hipLaunchKernelGGL((k_stage<BI, BJ, BK, NV, W9, LIM_VANLEER>), g, dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((k_stage<BI, BJ, BK, NV, W9, LIM_MC>), g, dim3(NT), 0, s, a);
    } else {
        if (limiter == LIM_MINMOD) hipLaunchKernelGGL((k_stage<BI, BJ, BK, NV, 2, LIM_MINMOD>), g, dim3(NT), 0, s, a);
        else if (limiter == LIM_VANLEER)
            hipLaunchKernelGGL((k_stage<BI, BJ, BK, NV, 2, LIM_VANLEER>), g, dim3(NT), 0, s, a);
        else if (waves == 1) hipLaunchKernelGGL((k_stage<BI, BJ, BK, NV, 1, LIM_MC>), g, dim3(NT), 0, s, a);
        else hipLaunchKernelGGL((k_stage<BI, BJ, BK, NV, 2, LIM_MC>), g, dim3(NT), 0, s, a);
    }
}

#define IC_INSTANTIATE(BI, BJ, BK)                                                                  \
    template __global__ void k_stage<BI, BJ, BK, 8, 1, LIM_MC>(KArgs);                             \
    template __global__ void k_stage<BI, BJ, BK, 8, 2, LIM_MC>(KArgs);                             \
    template __global__ void k_stage<BI, BJ, BK, 8, 2, LIM_MINMOD>(KArgs);                         \
    template __global__ void k_stage<BI, BJ, BK, 8, 2, LIM_VANLEER>(KArgs);                        \
    template void launch_stage<BI, BJ, BK, 8>(dim3, hipStream_t, const KArgs &, int, int);         \
    template void launch_stage<BI, BJ, BK, 9>(dim3, hipStream_t, const KArgs &, int, int);

#include "shapes.inc"
#undef IC_INSTANTIATE
