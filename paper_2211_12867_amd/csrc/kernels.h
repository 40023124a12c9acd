// kernels.h -- HIP kernels of the Icarus hot path (gfx950).
//
// All kernels walk device-resident task lists with a grid-stride loop over
// work-groups, so a captured graph stays valid when a regrid rewrites the
// lists.  Block shapes are template parameters (BI x BJ x BK cells), and so
// is the number of conserved variables NV (8, or 9 with the CME density
// tracer).
#pragma once
#include "device.h"
#include "physics.h"

// Ghost-slab face geometry: tangential directions of face direction d, in
// increasing order.
__host__ __device__ constexpr int tan1(int d) { return d == 0 ? 1 : 0; }
__host__ __device__ constexpr int tan2(int d) { return d == 2 ? 1 : 2; }

struct KArgs {
    double *U;                 // state read by this kernel (stage input)
    const double *Ubase;       // U^n
    double *Uout;              // stage output
    const BlockDesc *desc;
    double *slabs;
    double *freg;
    const LevelGeo *geo;       // [IC_MAX_LEVEL + 2], index = level
    const MemberConst *mc;
    const int *items;          // work list (slots)
    const int *nitems;
    const double *dt;          // per member
    const double *t;           // per member
    double *rate;              // per slot
    int *bad;                  // per member: [2m] = 1 + slot of the first non-physical cell, [2m+1] = its cell
    unsigned long long *floors; // per member: [2m] cells the density floor acted on, [2m+1] the pressure floor
    long slab_stride;          // doubles per slab
    long reg_stride;           // doubles per flux register
    double alpha;              // stage weight of dt (1/2 or 1)
    double tfrac;              // stage time = t + tfrac * dt
    Gas gas;
    double omega, gm;
    double rho_floor, p_floor;
    int cart;
    int want_rate;
    int xcd_order;             // stage kernel: XCD-contiguous runs of the work list
    int ksplit;                // stage kernel: work-groups per block, each marching over BK / ksplit planes
    double *divb;              // parabolic cleaning: div B of the stage input per slot and cell
    double divb_cd;            // parabolic cleaning coefficient C_d (0 = off)
    int nv;                    // conserved variables per cell (8, or 9 with the tracer)
};

// CFL maxima are kept per block and k-part: rate[slot * KSPLIT_MAX + part]
// (a block of up to KSPLIT_MAX planes along phi can give each plane its own
// work-group)
#define KSPLIT_MAX 12

template <int BI, int BJ, int BK, int NV_ = 8>
struct Shape {
    static constexpr int B0 = BI, B1 = BJ, B2 = BK;
    static constexpr int NC = BI * BJ * BK;
    static constexpr int NV = NV_;              // conserved variables per cell
    __host__ __device__ static constexpr int dim(int d) { return d == 0 ? BI : (d == 1 ? BJ : BK); }
    __host__ __device__ static constexpr int face_cells(int d) { return dim(tan1(d)) * dim(tan2(d)); }
    static constexpr int MAXFACE = (BI * BJ > BI * BK ? (BI * BJ > BJ * BK ? BI * BJ : BJ * BK)
                                                       : (BI * BK > BJ * BK ? BI * BK : BJ * BK));
};

// Address of variable v of the cell (i, j, k) of block `slot`, where at most
// one index may lie in the two ghost layers: interior, same-level neighbour,
// outflow copy of the edge cell, or ghost slab.  Within a block or a slab the
// cells of one (i, j) plane are contiguous in i, then j.
template <class S>
__device__ inline const double *ghosted_addr(const double *__restrict__ U, const BlockDesc *__restrict__ desc,
                                             const double *__restrict__ slabs, long slab_stride, int slot, int v,
                                             int i, int j, int k)
{
    int idx[3] = {i, j, k};
    int d = -1;
    if (i < 0 || i >= S::B0) d = 0;
    else if (j < 0 || j >= S::B1) d = 1;
    else if (k < 0 || k >= S::B2) d = 2;
    if (d < 0) return U + (size_t)slot * S::NV * S::NC + (size_t)v * S::NC + i + S::B0 * (j + S::B1 * k);
    const int Bd = S::dim(d);
    const int side = idx[d] >= Bd ? 1 : 0;
    const int l = side ? idx[d] - Bd : idx[d] + 2;
    const int code = desc[slot].nbr[2 * d + side];
    if (code >= 0) {
        idx[d] = side ? l : Bd - 2 + l;
        return U + (size_t)code * S::NV * S::NC + (size_t)v * S::NC + idx[0] + S::B0 * (idx[1] + S::B1 * idx[2]);
    }
    if (code == NBR_OUTFLOW) {
        idx[d] = side ? Bd - 1 : 0;
        return U + (size_t)slot * S::NV * S::NC + (size_t)v * S::NC + idx[0] + S::B0 * (idx[1] + S::B1 * idx[2]);
    }
    const int s = nbr_slab(code);
    const int a = idx[tan1(d)], b = idx[tan2(d)];
    const int FA = S::dim(tan1(d)), FB = S::dim(tan2(d));
    return slabs + (size_t)s * slab_stride + ((size_t)(v * 2 + l) * FB + b) * FA + a;
}

// The six face codes of a block (BlockDesc::nbr), held in scalar registers.
struct Faces {
    int n0, n1, n2, n3, n4, n5;
};

// Face codes of block `slot` (the same for every lane of the work-group).
__device__ inline Faces load_faces(const BlockDesc *desc, int slot)
{
    const int *dn = desc[slot].nbr;
    return Faces{__builtin_amdgcn_readfirstlane(dn[0]), __builtin_amdgcn_readfirstlane(dn[1]),
                 __builtin_amdgcn_readfirstlane(dn[2]), __builtin_amdgcn_readfirstlane(dn[3]),
                 __builtin_amdgcn_readfirstlane(dn[4]), __builtin_amdgcn_readfirstlane(dn[5])};
}

DEV int face_code(const Faces &nb, int f)
{
    return f == 0 ? nb.n0 : f == 1 ? nb.n1 : f == 2 ? nb.n2 : f == 3 ? nb.n3 : f == 4 ? nb.n4 : nb.n5;
}

// Address of variable v of the cell (i, j, k) of block `slot`, where at most
// one index lies in the two ghost layers (interior, same-level neighbour,
// outflow copy of the edge cell or ghost slab), with the block's face codes
// in registers: the cases of ghosted_addr without a descriptor load per
// lane.  With i = j = 0 it gives the start of a k-plane, whose cells are
// contiguous in i, then j, in a block, a slab and an outflow copy.
template <class S>
DEV const double *cell_addr(const double *__restrict__ U, const double *__restrict__ slabs, long slab_stride,
                            int slot, const Faces &nb, int v, int i, int j, int k)
{
    int idx[3] = {i, j, k};
    int d = -1;
    if (i < 0 || i >= S::B0) d = 0;
    else if (j < 0 || j >= S::B1) d = 1;
    else if (k < 0 || k >= S::B2) d = 2;
    if (d < 0) return U + (size_t)slot * S::NV * S::NC + (size_t)v * S::NC + i + S::B0 * (j + S::B1 * k);
    const int Bd = S::dim(d);
    const int side = idx[d] >= Bd ? 1 : 0;
    const int l = side ? idx[d] - Bd : idx[d] + 2;
    const int code = face_code(nb, 2 * d + side);
    if (code >= 0) {
        idx[d] = side ? l : Bd - 2 + l;
        return U + (size_t)code * S::NV * S::NC + (size_t)v * S::NC + idx[0] + S::B0 * (idx[1] + S::B1 * idx[2]);
    }
    if (code == NBR_OUTFLOW) {
        idx[d] = side ? Bd - 1 : 0;
        return U + (size_t)slot * S::NV * S::NC + (size_t)v * S::NC + idx[0] + S::B0 * (idx[1] + S::B1 * idx[2]);
    }
    const int a = idx[tan1(d)], b = idx[tan2(d)];
    const int FA = S::dim(tan1(d)), FB = S::dim(tan2(d));
    return slabs + (size_t)nbr_slab(code) * slab_stride + ((size_t)(v * 2 + l) * FB + b) * FA + a;
}

template <class S>
__device__ inline double ghosted(const double *__restrict__ U, const BlockDesc *__restrict__ desc,
                                 const double *__restrict__ slabs, long slab_stride, int slot, int v,
                                 int i, int j, int k)
{
    return *ghosted_addr<S>(U, desc, slabs, slab_stride, slot, v, i, j, k);
}

// Refinement criteria: the Sect. 3.2 shock criterion, the Sect. 3.1 tracer
// criterion, and their union inside the windows (Sect. 3.3).
enum { CRIT_SHOCK = 0, CRIT_TRACER = 1, CRIT_COMBINED = 2 };

struct IndicatorParams {
    int max_level;
    double eps, tol_r, tol_c, w_rho, w_v;
    int use_windows;
    double lon_e, clt_e, dlon_e, dclt_e, dlon_c;   // radians
    int criterion;                                 // CRIT_*
    double tr_r, tr_c;                             // tracer fractions that refine / keep a block
};

// Launch wrappers per block shape (kernels.hip, stage.hip); the runtime calls these.
struct Launchers {
    void (*stage)(dim3, hipStream_t, const KArgs &, int waves, int limiter);
    void (*hancock)(dim3, hipStream_t, const KArgs &, int limiter);
    void (*divb)(dim3, hipStream_t, const KArgs &);
    void (*clean)(dim3, hipStream_t, const KArgs &);
    void (*slabs)(dim3, hipStream_t, const KArgs &, const SlabTask *, const int *, int pass);
    void (*reflux)(dim3, hipStream_t, const KArgs &, const RefluxTask *, const int *, const int *);
    void (*rate)(dim3, hipStream_t, const KArgs &);
    void (*indicator)(dim3, hipStream_t, const KArgs &, int8_t *, const IndicatorParams &);
    void (*move)(dim3, hipStream_t, const KArgs &, double *, const MoveTask *, int);
    void (*sample)(dim3, hipStream_t, const KArgs &, const SampleDesc *, int, double *, double *, int *, int, int,
                   double *, long *);
};
bool get_launchers(int bi, int bj, int bk, int nv, Launchers *out);
void launch_dt(hipStream_t s, const KArgs &a, const int *mbeg, const int *mend, int nm, double cfl,
               double dt_fixed, const double *tend, double *dt_last);
void launch_time(hipStream_t s, double *t, const double *dt, long *nsteps, int nm);

// kernel entry points (stage.hip: k_stage and its launcher; kernels.hip: the rest)
template <int BI, int BJ, int BK, int NV, int W, int LIM> __global__ void k_stage(KArgs a);
template <int BI, int BJ, int BK, int NV> void launch_stage(dim3 g, hipStream_t s, const KArgs &a, int waves, int limiter);
template <int BI, int BJ, int BK, int NV, int LIM> __global__ void k_hancock(KArgs a);
template <int BI, int BJ, int BK, int NV> __global__ void k_divb(KArgs a);
template <int BI, int BJ, int BK, int NV> __global__ void k_clean(KArgs a);
template <int BI, int BJ, int BK, int NV> void launch_hancock(dim3 g, hipStream_t s, const KArgs &a, int limiter);
template <int BI, int BJ, int BK, int NV, int PASS>
__global__ void k_slabs(KArgs a, const SlabTask *tasks, const int *range);
template <int BI, int BJ, int BK, int NV>
__global__ void k_reflux(KArgs a, const RefluxTask *tasks, const int *ranges, const int *ntasks);
template <int BI, int BJ, int BK, int NV> __global__ void k_rate(KArgs a);
template <int BI, int BJ, int BK, int NV>
__global__ void k_indicator(KArgs a, int8_t *flags, IndicatorParams p);
template <int BI, int BJ, int BK, int NV>
__global__ void k_move(KArgs a, double *Unew, const MoveTask *tasks, int ntasks);
template <int BI, int BJ, int BK, int NV>
__global__ void k_sample(KArgs a, const SampleDesc *sd, int nmembers, double *out, double *ring,
                         int *ring_count, int ring_cap, int record, double *t_step, long *nsteps);

__global__ void k_dt(KArgs a, const int *mbeg, const int *mend, int nmembers, double cfl,
                     double dt_fixed, const double *tend, double *dt_last);
__global__ void k_time(double *t, const double *dt, long *nsteps, int nmembers);
