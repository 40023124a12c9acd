// device.h -- data layouts shared by the host runtime and the HIP kernels.
//
// Memory in HBM (one allocation each, fixed capacity for the sim's lifetime so
// that captured graphs stay valid across regrids):
//   U, Us        state and stage buffer, [slot][var][k][j][i] fp64 (SoA per block,
//                i = r fastest); slot = member * max_blocks + local slot
//   slabs        ghost slabs for faces that are not same-level neighbours and
//                not outflow: [slab][var][layer][b][a], 2 layers
//   fluxreg      raw face fluxes at coarse-fine faces: [reg][var][b][a]
//   desc         BlockDesc per slot
//   geo          per-level 1-D metric tables (RecR / RecT / RecP)
//   task lists   work items of each kernel, counts in device memory
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define IC_NV 8
#define IC_MAX_LEVEL 6
#define IC_NG 2

// neighbour codes in BlockDesc::nbr
#define NBR_OUTFLOW (-1)
// slab s is encoded as -(s + 2)
__host__ __device__ inline int nbr_slab(int code) { return -code - 2; }
__host__ __device__ inline int slab_code(int s) { return -s - 2; }

struct BlockDesc {
    int level;        // 1-based
    int member;
    int org[3];       // global cell index of the block's first cell on its level
    int nbr[6];       // face (d, side) -> 2*d+side: same-level slot >= 0, NBR_OUTFLOW, or slab code
    int freg[6];      // flux register for the face, -1 if none
    int reflux_mask;  // bit f set: the block is the coarse side at face f (its edge cells get refluxed)
    int pad;
};

// Radial (or x) metric record of cell m on a level, stored at index m + 2.
struct RecR {
    double idm, idp, idc;   // 1/(x_m - x_{m-1}), 1/(x_{m+1} - x_m), 1/(x_{m+1} - x_{m-1}), x = centres
    double hm, hp;          // x_m - f_m, f_{m+1} - x_m
    double am, ap;          // A_r/V at the lower / upper face (angular factors cancelled)
    double rt;              // 1/r in finite-volume form (1 for cartesian)
    double rc;              // centre
    double icfl;            // 1/dr
    double irc;             // 1/r_c (1 for cartesian)
    double vw;              // radial factor of the volume
    double poff;            // x_m - centroid of the two children of m's parent (prolongation)
    double r2f;             // radial factor of A_r at the lower face
    double r2h;             // radial factor of A_theta and A_phi
    double pad;
};

// Colatitude (or y) metric record.
struct RecT {
    double idm, idp, idc, hm, hp;
    double thm, thp;        // sin(theta_-)/dmu, sin(theta_+)/dmu (1/dy cartesian)
    double ctil;            // cot(theta) in finite-volume form
    double sinc, cosc;      // of the centre
    double phf;             // dtheta/dmu (1 cartesian); phi metric = rt * phf * RecP::iw
    double icfl;            // 1/dtheta
    double isinc;           // 1/sin(theta_c) (1 cartesian)
    double vw;              // dmu = cos t- - cos t+  (dy cartesian)
    double poff;
    double sf;              // angular factor of A_theta at the lower face: sin(theta_f) (1 cartesian)
    double dth;             // angular factor of A_phi: dtheta (dy cartesian)
    double tc;              // centre
};

// Longitude (or z) metric record.
struct RecP {
    double idm, idp, idc, hm, hp;
    double iw;              // 1/dphi
    double vw;              // dphi
    double poff;
    double pc;              // centre
};

struct LevelGeo {
    const RecR *r;          // n_r + 4 records
    const RecT *t;
    const RecP *p;
    int n[3];               // cells on this level
    int pad;
    const double *wind;     // inner-boundary wind primitives [6][n_t][n_p]: rho, v_r, v_phi, p, B_r, B_phi
    const double *cosd;     // cos of the CME distance per member: [member][n_t][n_p]
};

// Per-member constants.
struct MemberConst {
    // cone CME (code units): active when 0 <= t - t0 <= tact
    double t0, tact, v, r_half, rho, p;
    int enabled;
    int pad;
    double lon_cme;         // radians (refinement window)
    double r_in;            // inner boundary radius
};

// Ghost-slab fill task.
enum { SLAB_INNER = 0, SLAB_RESTRICT = 1, SLAB_PROLONG = 2 };
struct SlabTask {
    int type;
    int slab;
    int slot;               // owner block
    int face;               // 2*d + side of the owner
    int src[4];             // RESTRICT: fine slots by quadrant qa + 2 qb; PROLONG: src[0] coarse slot
    int shift[3];           // RESTRICT: owner-level index wrap shift per direction;
                            // PROLONG: coarse local = floor(g/2) + shift
    int fbase[3];           // RESTRICT: fine block index of quadrant 0 per direction
    int cwrap[3];           // PROLONG: coarse global (wrapped) = floor(g/2) + cwrap
    int pad;
};

// Reflux task: one coarse face of a block with four finer neighbours.
struct RefluxTask {
    int slot;               // coarse block
    int face;
    int creg;               // coarse block's own flux register at the face
    int freg[4];            // fine blocks' registers by quadrant qa + 2 qb
    int last;               // 1 on the block's last task (rate refresh)
};

// Regrid data move.
enum { MOVE_PROLONG = 0, MOVE_RESTRICT = 1 };
struct MoveTask {
    int type;
    int dst;                // new slot
    int src[8];             // PROLONG: src[0] parent slot, src[1] child octant; RESTRICT: 8 children by octant
    int level;              // level of dst
    int org[3];             // dst origin (cells, on its level)
};

// Sample stencil entry.
struct SampleEntry {
    double w;
    int kind;               // 0: one cell; 1: volume-weighted mean of 8 children
    int slot;
    int cell[3];            // local cell (kind 0) or local first child (kind 1)
    int level;              // level of the cells read
    int g[3];               // global index of the first child (kind 1) for weights
};

struct SampleDesc {
    SampleEntry e[8];
    int valid;
    int pad;
};
