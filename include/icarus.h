/*
 * icarus.h -- C ABI of the MI355X library for the Icarus hot path.
 *
 * The library advances 3-D ideal MHD in the frame co-rotating with the Sun on
 * a spherical (r, theta, phi) grid with radial stretching and block-adaptive
 * refinement (Baratashvili et al., "Improving CME evolution and arrival
 * predictions with AMR and grid stretching in Icarus", Sect. 2.1-2.2, 3):
 * a finite-volume TVDLF (Rusanov) scheme with a monotonised-central limiter,
 * second order in space and time, two ghost layers, inner-boundary driving by
 * a solar wind plus a cone CME (Eqs. 1-4), refinement by a Loehner-type
 * density/velocity indicator restricted to compressive cells (div V < 0)
 * inside the Earth/CME windows of Sect. 3.2.
 *
 * Conventions
 *  - Every pointer argument is a plain host pointer unless it says "device".
 *    Config structs are copied during ic_create; output buffers belong to the
 *    caller.  The sim object and all device memory it uses belong to the
 *    library and are released by ic_destroy.
 *  - Units at the ABI: AU, degrees, seconds, km/s, cm^-3, K, nT, m^3/s^2.
 *    State arrays (ic_get_state / ic_set_state / sampled primitives) are in
 *    the library's code units: length 1 AU, speed 1000 km/s, time
 *    1 AU / (1000 km/s), density m_p cm^-3, pressure and energy density
 *    rho0 v0^2, magnetic field sqrt(mu0 rho0 v0^2) (mu0 = 1); ic_units()
 *    returns these scales.
 *  - Conserved variables, 8 per cell: rho, m_r, m_theta, m_phi, E, B_r,
 *    B_theta, B_phi (x, y, z in the cartesian test geometry); 9 with the
 *    CME density tracer (ic_phys_cfg.tracer), the ninth being rho s.
 *  - Block state layout: [block][variable][k][j][i], i (r) fastest, blocks in
 *    ascending (level, Morton(i, j, k)) order, as ic_get_blocks lists them.
 *  - All GPU work is enqueued on the HIP stream given to ic_create (NULL =
 *    the null stream).  Calls that return host data synchronise that stream.
 *  - Errors: the return value is IC_OK or a negative ic_status; ic_last_error
 *    gives a text for the last failing call on the calling thread.  After
 *    IC_E_UNPHYSICAL, IC_E_DEVICE or IC_E_CAPACITY the sim is poisoned and
 *    every later call except ic_destroy returns IC_E_STATE.
 *  - One sim is used from one thread at a time.
 */
#ifndef ICARUS_H
#define ICARUS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ic_sim ic_sim;

typedef enum {
    IC_OK = 0,
    IC_E_INVALID = -1,     /* bad argument or configuration */
    IC_E_NOMEM = -2,       /* device or host allocation failed */
    IC_E_DEVICE = -3,      /* a HIP call failed */
    IC_E_UNPHYSICAL = -4,  /* rho <= 0, p <= 0 or a non-finite value in a leaf cell */
    IC_E_OUTSIDE = -5,     /* sample point outside the domain */
    IC_E_CAPACITY = -6,    /* block pool too small for the requested forest */
    IC_E_STATE = -7        /* the sim was poisoned by an earlier error */
} ic_status;

enum { IC_GEOM_SPHERICAL = 0, IC_GEOM_CARTESIAN = 1 };
enum { IC_BC_OUTFLOW = 0, IC_BC_PERIODIC = 1, IC_BC_INNER = 2 };
enum { IC_FLAG_COARSEN = -1, IC_FLAG_KEEP = 0, IC_FLAG_REFINE = 1 };

/* Mesh (Sect. 2.2, 3).  Spherical: x = (r [AU], colatitude [deg], longitude
 * [deg]); cartesian (tests): code units.  Level l has n * 2^(l-1) cells per
 * direction; blocks hold block[0] x block[1] x block[2] cells and block must
 * be one of the sizes the library is built for (ic_block_supported).
 * stretched_r = 1 gives radial faces r_in exp(k ln(r_out/r_in)/N_l) (cells
 * of equal aspect, Eq. 5); 0 gives equidistant faces.  bc[d][0/1]: lower /
 * upper boundary of direction d; IC_BC_INNER is the wind + CME inner
 * boundary (spherical r lower side only); periodic needs both sides periodic.
 * max_blocks: block-pool capacity per member (0 = a default). */
typedef struct {
    int geometry;
    double x0[3], x1[3];
    int n[3];
    int block[3];
    int stretched_r;
    int max_level;
    int bc[3][2];
    int max_blocks;
} ic_grid_cfg;

/* Physics: adiabatic index, CFL number (dt = cfl / max sum_d (|v_d|+c_f)/dx_d),
 * frame rotation rate [rad/s] about the theta = 0 axis, G M_sun [m^3 s^-2],
 * small-value floors in code units applied to every stage result (a cell with
 * rho < rho_floor takes rho_floor at zero velocity; then a cell with
 * p < p_floor has its energy raised to give p = p_floor; 0 disables).
 * Scheme (Sect. 2.1: TVDLF with the Woodward limiter in the paper's runs; its
 * code offers other scheme and limiter combinations): limiter of the
 * primitive reconstruction, IC_LIM_MC (monotonised central, the Woodward
 * form; the default), IC_LIM_MINMOD or IC_LIM_VANLEER (harmonic mean of the
 * one-sided differences); scheme IC_SCHEME_TWO_STAGE (U* = U^n + dt/2 L(U^n),
 * U^{n+1} = U^n + dt L(U*); the default) or IC_SCHEME_HANCOCK (the one-step
 * TVDLF: the predictor U* = U^n + dt/2 L_H(U^n) takes each cell's own physical
 * fluxes at its reconstructed face states, no interface solver, then the same
 * conservative second stage).  divb_cd > 0 turns on the parabolic div B
 * cleaning the paper applies (Sect. 2.1), off by default: after each stage
 * (reflux and floors included) B += alpha divb_cd h^2 grad(div B) with alpha
 * the stage weight (1/2, 1), div B of the stage input in face-mean form,
 * central differences between face neighbours in physical components,
 * h^2 = 1 / sum_d dx_d^-2 (the CFL widths), and E += B_in . dB; no gradient
 * component across a physical boundary or a level change; divb_cd in [0, 1]
 * (a Fourier mode decays by 1 - alpha divb_cd (h/dx)^2 sin^2(k dx) per
 * application).  tracer = 1 carries the CME density tracer of Sect. 3.1 as a
 * ninth conserved variable rho s (s the CME mass fraction: 1 in the cone CME
 * at the inner boundary, 0 in the wind and in the initial state), advected
 * by the same TVDLF flux with the same maximum speed, no source, left alone
 * by the floors; with any limiter and either time scheme. */
enum { IC_LIM_MC = 0, IC_LIM_MINMOD = 1, IC_LIM_VANLEER = 2 };
enum { IC_SCHEME_TWO_STAGE = 0, IC_SCHEME_HANCOCK = 1 };
typedef struct {
    double gamma;
    double cfl;
    double omega;
    double gm;
    double rho_floor;
    double p_floor;
    int limiter;
    int scheme;
    double divb_cd;
    int tracer;
} ic_phys_cfg;

/* Inner-boundary wind at r_in (Sect. 2.1): v_r = v_min + (v_max - v_min)
 * (f - f_min)/(f_max - f_min), clamped, f = sum a_lm Y_lm(theta, phi) over
 * l = 1..3 (orthonormal real harmonics, no Condon-Shortley phase, (l, m)
 * order); v_r = v_min everywhere if f_max <= f_min.  n = n_ref (v_r/v_ref)^-2,
 * p = 2 n k_B T, v_phi = -omega r_in sin(theta), B a unipolar Parker field of
 * magnitude B_nT parallel to v in the co-rotating frame. */
typedef struct {
    double alm[15];
    double f_min, f_max;
    double v_min_kms, v_max_kms;
    double n_ref_cm3, v_ref_kms;
    double T_K;
    double B_nT;
} ic_wind_cfg;

/* Cone CME (Eqs. 1-4): inner-boundary points with angular distance d to the
 * CME centre below the opening angle theta(t) take n, T, v_r = v_kms (B and
 * v_phi of the wind), for 0 <= t - t_start <= min(duration, 2 r_1/2 / v). */
typedef struct {
    double t_start_s, duration_s, v_kms, half_width_deg, colat_deg, lon_deg, n_cm3, T_K;
    int enabled;
} ic_cme_cfg;

/* Refinement criterion (Sect. 3.2 windows): a cell is hot at tolerance tol if
 * it lies in |lon - lon_E| <= dlon_E, |colat - colat_E| <= dclt_E and
 * |lon - lon_CME| <= dlon_CME (when use_windows), has div V < 0 and
 * w_rho E(rho) + w_v E(|v|) > tol, E the per-direction Loehner estimator
 * with parameter eps_lohner.  A block is REFINE below max_level with a hot
 * cell at tol_refine, COARSEN above level 1 with no hot cell at tol_coarsen,
 * else KEEP.  buffer_blocks = 1 refines the face neighbours of REFINE blocks
 * too.  regrid_every is the cadence ic_advance regrids at (0 = never).
 * criterion: IC_CRIT_SHOCK (the above, Sect. 3.2; the default),
 * IC_CRIT_TRACER (Sect. 3.1: a cell is hot where the tracer fraction
 * s = (rho s) / rho exceeds tracer_refine, resp. tracer_coarsen, anywhere,
 * without windows) or IC_CRIT_COMBINED (Sect. 3.3: a cell inside the windows
 * is hot by either condition); the latter two need the tracer and the plain
 * source.  The learned flags and ic_eval_hot follow the shock criterion. */
enum { IC_CRIT_SHOCK = 0, IC_CRIT_TRACER = 1, IC_CRIT_COMBINED = 2 };
typedef struct {
    double eps_lohner, tol_refine, tol_coarsen, w_rho, w_v;
    double lon_earth_deg, clt_earth_deg, dlon_earth_deg, dclt_earth_deg, dlon_cme_deg;
    int use_windows;
    int regrid_every;
    int buffer_blocks;
    int source;             /* IC_SOURCE_*: where ic_regrid(sim, NULL, ...) takes its flags from */
    int judge_every;        /* learned + judge: evaluate the plain criterion every judge_every-th regrid */
    double judge_recall;    /* fall back to the plain flags for 10 regrids below this REFINE recall */
    double learned_threshold; /* learned REFINE where the network's p >= this (<= 0: 1/2) */
    int criterion;          /* IC_CRIT_* */
    double tracer_refine, tracer_coarsen;   /* tracer fractions (tracer and combined criteria) */
} ic_amr_cfg;

enum { IC_SOURCE_PLAIN = 0, IC_SOURCE_LEARNED = 1, IC_SOURCE_LEARNED_JUDGED = 2 };

typedef struct {
    long steps;              /* steps taken by member 0 since ic_create */
    double t_s;              /* time of member 0 */
    double dt_s;             /* last step of member 0 */
    double zone_updates;     /* leaf cells advanced by full steps, all members, since ic_create */
    int leaves;              /* leaf blocks of member 0 */
    int leaves_per_level[8];
} ic_info;

/* Create a sim of n_members independent runs sharing one grid and wind,
 * member m driven by cmes[m] (cmes may be NULL: no CME).  The state starts
 * from the relaxation initial condition: rho ~ r^-2, v_r constant along
 * rays, p ~ r^-2 gamma, B_r ~ r^-2, v_phi = -omega r sin(theta) and B
 * parallel to v.  amr may be NULL when max_level = 1.  hip_stream is a
 * hipStream_t (NULL = null stream).  On success *out owns the sim. */
ic_status ic_create(const ic_grid_cfg *grid, const ic_phys_cfg *phys, const ic_wind_cfg *wind,
                    const ic_cme_cfg *cmes, int n_members, const ic_amr_cfg *amr,
                    void *hip_stream, ic_sim **out);

/* Release the sim and its device memory (NULL is ignored). */
void ic_destroy(ic_sim *sim);

/* One two-stage step of every member (paper Sect. 2.1: second order in time):
 * U* = U^n + dt/2 L(U^n) with ghosts at t^n, U^{n+1} = U^n + dt L(U*) with
 * ghosts at t^n + dt/2.  dt_fixed_s > 0 forces dt; 0 takes the CFL dt of
 * each member.  out may be NULL.  Returns IC_E_UNPHYSICAL (sim poisoned) if
 * a stage input or the step's result holds rho <= 0, p <= 0 or a
 * non-finite value in a leaf cell. */
ic_status ic_step(ic_sim *sim, double dt_fixed_s, ic_info *out);

/* Time evolution with solution-driven refinement (Sect. 2.1, 3): advance
 * every member by dt_s (the last step is clipped to land on t + dt_s), at most
 * max_steps steps, recording the sample point after every step
 * (ic_timeseries).  When max_level > 1 the forest is rebuilt by the plain or
 * learned criterion (amr->source) after every amr->regrid_every steps; the
 * count runs across calls (steps taken by ic_step count too, any regrid
 * restarts it), so advancing in pieces regrids after the same steps as one
 * advance over the whole span.  Returns IC_E_UNPHYSICAL (sim poisoned) if a
 * stage input or a step's result holds rho <= 0, p <= 0 or a non-finite
 * value. */
ic_status ic_advance(ic_sim *sim, double dt_s, long max_steps, ic_info *out);

/* Rebuild every member's forest (Sect. 3): flags NULL evaluates the plain
 * criterion on the current state; otherwise flags[m * max_blocks + b] gives
 * member m's flag for its b-th leaf in ic_get_blocks order (IC_FLAG_*).
 * Then buffer, 2:1 closure over all 26 neighbours, coarsening of complete
 * sibling octets, and data movement by conservative limited prolongation /
 * volume-weighted restriction.  Returns IC_E_CAPACITY (sim poisoned) if the
 * pool cannot hold the new forest. */
ic_status ic_regrid(ic_sim *sim, const int8_t *flags, ic_info *out);

/* Plain-criterion flags of member's leaves, in ic_get_blocks order; n is the
 * capacity of flags and must be >= the leaf count. */
ic_status ic_eval_flags(ic_sim *sim, int member, int8_t *flags, int n);

/* Refinement condition without the level cap (Sect. 3.2 criterion): hot[q] = 1
 * if some cell of leaf q (ic_get_blocks order) lies in the windows, is
 * compressive and has an indicator above tol_refine, else 0, whatever the
 * leaf's level.  Look-ahead labels for the learned flags are built from it.
 * n is the capacity of hot and must be >= the leaf count. */
ic_status ic_eval_hot(ic_sim *sim, int member, int8_t *hot, int n);

/* Refinement windows per leaf (ic_get_blocks order): in[q] = 1 if some cell
 * centre of leaf q lies in the Sect. 3.2 windows of the member (always 1 with
 * use_windows = 0).  Learned flags ask for refinement only on such leaves. */
ic_status ic_eval_window(ic_sim *sim, int member, int8_t *in, int n);

/* Time series at Earth (Sect. 3.1 compares the runs by the solar-wind
 * variables recorded at Earth): primitive variables (rho, v_r, v_theta,
 * v_phi, p, B_r, B_theta, B_phi), code units, at a point: trilinear interpolation between the cell centres of the
 * level of the finest leaf containing the point (cells of a coarser leaf
 * count with their covering value, cells under finer leaves with the
 * volume-weighted mean of their children).  IC_E_OUTSIDE outside the domain. */
ic_status ic_sample(ic_sim *sim, int member, double r_au, double colat_deg, double lon_deg,
                    double prim_out[8]);

/* Point recorded after every step by ic_advance and ic_step (default (1 AU,
 * 90, 0): Earth in the co-rotating frame, Sect. 3.1). */
ic_status ic_set_sample_point(ic_sim *sim, double r_au, double colat_deg, double lon_deg);

/* Recorded time series at the sample point (Sect. 3.1), one entry per step
 * a member took (a step past its end time, dt = 0, records nothing):
 * out[s * 9 + 0] = t [s], out[s * 9 + 1..8] =
 * primitives (code units); *n_inout is the capacity in samples on entry and
 * the count written on return (the most recent ones if the record is longer).
 * ic_timeseries_clear drops the record. */
ic_status ic_timeseries(ic_sim *sim, int member, double *out, int *n_inout);
ic_status ic_timeseries_clear(ic_sim *sim);

/* Leaf blocks of a member as (level, i, j, k) quadruples, level >= 1, in
 * ascending (level, Morton) order.  *n_inout: capacity on entry (in blocks),
 * leaf count on return; IC_E_INVALID if the capacity is too small. */
ic_status ic_get_blocks(ic_sim *sim, int member, int32_t *lvl_ijk, int *n_inout);

/* Copy a member's conserved state (the finite-volume cell averages of the
 * eight conserved MHD variables, Sect. 2.1, then rho s with the tracer) to
 * host_U ([block][nv][bk][bj][bi], nv = 8 or 9, code units, blocks in
 * ic_get_blocks order); n_doubles must be >= leaves * nv * cells per block.
 * Synchronises the stream. */
ic_status ic_get_state(ic_sim *sim, int member, double *host_U, size_t n_doubles);

/* Replace a member's block forest (Sect. 3: blocks of 2:1-balanced levels)
 * and state: n_blocks leaves (level, i, j, k) that tile the domain without
 * overlap and keep 2:1 balance, with data host_U in the ic_get_state layout,
 * at time t_s (a checkpoint restart).  IC_E_INVALID for a forest that does
 * not tile or balance, IC_E_CAPACITY beyond the pool.  The regrid step count
 * restarts; the floor counts are kept. */
ic_status ic_set_state(ic_sim *sim, int member, const int32_t *lvl_ijk, int n_blocks,
                       const double *host_U, double t_s);

/* Time and last dt of a member [s]. */
ic_status ic_get_time(ic_sim *sim, int member, double *t_s, double *dt_s);

/* Checkpoint clock (the paper starts its CME runs from a saved relaxed wind,
 * Sect. 2.1 and 3.1): the member's time in code units exactly as the library
 * holds it, and the steps ic_advance has taken since the last regrid (one
 * count per sim, shared by the members).  ic_set_state takes its time in
 * seconds, and t * T0 does not always convert back to the same double; a
 * restart that must continue bit for bit calls ic_set_clock after
 * ic_set_state (which restarts the regrid count) with the values
 * ic_get_clock gave at the checkpoint.  IC_E_INVALID for a non-finite time
 * or a negative count.  Both synchronise the stream. */
ic_status ic_get_clock(ic_sim *sim, int member, double *t_code, long *since_regrid);
ic_status ic_set_clock(ic_sim *sim, int member, double t_code, long since_regrid);

/* Small-value floors acted on (the paper's scheme is not positivity
 * preserving and it does not say how small values are treated; see
 * ic_phys_cfg): the number of cell updates of a member since ic_create at
 * which the density floor (*rho_floors) and the pressure floor (*p_floors)
 * changed the state, counted in every stage.  Either pointer may be NULL.
 * Synchronises the stream. */
ic_status ic_floor_counts(ic_sim *sim, int member, long *rho_floors, long *p_floors);

/* Shock diagnostics of a radial-speed series at a point (Sect. 3.1: arrival
 * time and shock width, measured from the arrival to the peak speed once the
 * speed has jumped; Sect. 3.2: peak speed and average gradient of the
 * shock).  t_s[n] ascending sample times [s], v[n] the speeds
 * (any unit), t_cme_s the CME start, window_s the span after it searched for
 * the peak, min_jump the smallest rise (unit of v) counted as a shock.
 * v_pre = v at t_cme_s (linear between samples), v_max = the largest sample
 * in [t_cme_s, t_cme_s + window_s] (the first of equal ones; the peak speed),
 * arrival = the first upward crossing of v_pre + (v_max - v_pre)/2 inside
 * the window by a segment that starts at or after t_cme_s, linear between
 * samples; the top of the jump = the first sample from the end of that
 * segment on after which v no longer rises (or the window's last sample).  out[0]
 * arrival - t_cme_s [s], out[1] width = t(top) - arrival [s], out[2] v_pre,
 * out[3] v_max, out[4] average gradient (v_top - level at arrival) / width
 * [unit of v per s], out[5] t(top) [s], out[6] v_top, out[7] t(v_max) [s].
 * out[0], out[1], out[4], out[5], out[6] are NaN without an arrival (no
 * crossing, or v_max - v_pre < min_jump).  Host computation on plain arrays
 * (ic_timeseries gives v_r in column 2); IC_E_INVALID for null pointers,
 * n < 0 or times out of order. */
ic_status ic_shock_diagnostics(const double *t_s, const double *v, int n, double t_cme_s, double window_s,
                               double min_jump, double out[8]);

/* ---- learned refinement flags -------------------------------------------
 * A per-block network predicts whether the plain criterion will ask for
 * refinement: input 512 values = 8 primitives (log10 rho, v_r, v_theta, v_phi,
 * log10 p, B_r, B_theta, B_phi; code units) averaged over the cells of each of
 * the 4 x 4 x 4 sub-cubes of the block, order [primitive][k][j][i], z-scored
 * per input with training statistics; layers 512 -> 128 -> 128 -> 1, ReLU,
 * sigmoid; weights, inputs and hidden activations in bf16 with fp32
 * accumulation; p >= 1/2 means REFINE, otherwise the block may coarsen.
 * Parameter vector (fp32, IC_MLP_NPARAM values): W1[512][128] (input-major),
 * b1[128], W2[128][128], b2[128], w3[128], b3. */
#define IC_MLP_IN 512
#define IC_MLP_NPARAM 82305

typedef struct {
    int epochs, batch;
    float lr, beta1, beta2, eps;
    unsigned seed;           /* shuffling */
    float pos_weight;        /* <= 0: N_neg / N_pos of the training set */
} ic_mlp_hparams;

/* Un-normalised inputs of a member's leaves (ic_get_blocks order) into
 * raw[n x 512] fp32; block dims must be multiples of 4. */
ic_status ic_features(ic_sim *sim, int member, float *raw, int n);

/* Install a trained network (params fp32, per-input mean and std). */
ic_status ic_mlp_set(ic_sim *sim, const float *params, const float *mean, const float *std);

/* Network probability and flag per leaf: IC_FLAG_REFINE if p >= the threshold
 * (ic_amr_cfg.learned_threshold, default 1/2) and the
 * leaf touches the refinement windows (ic_eval_window), else IC_FLAG_COARSEN. */
ic_status ic_eval_learned(ic_sim *sim, int member, float *prob, int8_t *flags, int n);

/* Learned-flag bookkeeping since ic_create: regrids that used the network,
 * regrids judged, judged regrids that fell back, and the last judged REFINE
 * recall of member 0. */
ic_status ic_regrid_stats(ic_sim *sim, long *learned, long *judged, long *fallbacks, double *last_recall);

/* Train on n rows (raw inputs as ic_features gives them, labels 0/1) with
 * weighted binary cross-entropy and Adam on fp32 master weights, fwd/bwd on
 * the GPU.  params: initial values in, trained values out; mean/std out;
 * loss_per_epoch (may be NULL) gets the mean loss of each epoch.  Runs on the
 * null stream of the current device. */
ic_status ic_mlp_train(const float *raw, const uint8_t *y, long n, const ic_mlp_hparams *hp, float *params,
                       float *mean, float *std, float *loss_per_epoch);

/* Network probabilities of n rows of raw inputs (as ic_features gives them):
 * z-scored with mean/std, then the bf16 MFMA forward pass.  Runs on the null
 * stream of the current device. */
ic_status ic_mlp_infer(const float *raw, long n, const float *params, const float *mean, const float *std,
                       float *prob);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * probabilities of ic_mlp_infer with every array on the device and no
 * allocation of any kind.  raw_dev [n x 512], params_dev [IC_MLP_NPARAM],
 * mean_dev and std_dev [512] (std must be positive; the values are not
 * checked on the host), prob_dev [n]: device pointers owned by the caller.
 * The work is enqueued on hip_stream (NULL = the null stream) and the call
 * returns without synchronising; prob_dev is valid once the stream has
 * completed it.  Intermediate values live in a fixed device scratch of the
 * library (one copy per device, about 6.2 MiB, held until the process
 * ends), so n may not exceed IC_MLP_NOALLOC_ROWS (IC_E_INVALID).  Every call
 * on a device shares that scratch: calls that overlap on one device (other
 * streams, other threads) race and must be ordered by the caller.  Results
 * equal ic_mlp_infer's bit for bit. */
#define IC_MLP_NOALLOC_ROWS 4096
ic_status ic_mlp_infer_noalloc(const float *raw_dev, long n, const float *params_dev, const float *mean_dev,
                               const float *std_dev, float *prob_dev, void *hip_stream);

/* One forward and backward pass on n rows of already normalised inputs
 * (fp32, rounded to bf16 inside): gradient of the mean weighted BCE in
 * params layout, and the loss. */
ic_status ic_mlp_grad(const float *xnorm, const uint8_t *y, int n, float pos_weight, const float *params,
                      float *grad, float *loss);

/* Stage-kernel schedule.  None of these choices changes any result bit:
 * waves_per_simd (1 or 2) is the occupancy the kernel's register allocation
 * targets, grid the launch size (0 = one work-group per leaf block, else a
 * persistent grid striding over the work list), xcd_order = 1 lays the work
 * list out as 8 contiguous runs, one per XCD, so that neighbouring blocks
 * share an L2, ksplit (1 .. 12, at most BK) gives each block that many
 * work-groups, each marching over about BK / ksplit planes (for work lists too
 * short to fill the GPU; the face shared by two parts is computed by both from
 * the same inputs).
 * stage_ms / default_ms: measured mean stage time of the choice and of
 * (2, 0, 0, 1); from_cache: taken from the cache file; candidates: the
 * schedules timed. */
typedef struct {
    int waves_per_simd;
    int grid;
    int xcd_order;
    double stage_ms, default_ms;
    int from_cache;
    int candidates;
    int ksplit;
} ic_tune_info;

/* Pick the stage-kernel schedule for this sim: look the key (device, CU count,
 * block shape, variable count, work-item count to a power of two) up in
 * cache_path (a text file, one result per line; NULL = no cache), else time
 * every candidate on the current state (reps launches each; the state is not
 * changed) and append the winner to the cache (candidates within 1 % of the
 * best so far keep the earlier one; XCD-contiguous order is tried first; one
 * wave per SIMD is tried only while the launch has fewer than two work-groups
 * per CU).  The
 * choice applies to later steps; out may be NULL.  The sim remembers the result for this work-list
 * size (and reads the cache's results for other sizes): after each regrid the
 * schedule of the new size is used, or, for a size without one, two waves per
 * SIMD, one work-group per work item and the smallest k-split giving at least
 * 512 work-groups.  Without any tuning call that rule applies from the start. */
ic_status ic_autotune(ic_sim *sim, const char *cache_path, int reps, ic_tune_info *out);

/* Force a schedule (waves_per_simd, grid, xcd_order, ksplit of *tune); it is
 * kept across regrids until the next ic_autotune. */
ic_status ic_set_tuning(ic_sim *sim, const ic_tune_info *tune);

/* The schedule in force (waves_per_simd, grid, xcd_order, ksplit; the other
 * fields are zero). */
ic_status ic_get_tuning(ic_sim *sim, ic_tune_info *tune);

/* Code-unit scales in SI: [0] length m, [1] speed m/s, [2] time s, [3]
 * density kg/m^3, [4] pressure Pa, [5] field T. */
void ic_units(double out[6]);

/* Block-pool capacity per member (the stride of the flags array of ic_regrid). */
int ic_pool_capacity(const ic_sim *sim);

/* Device memory from the caller (for callers whose framework owns device
 * memory, e.g. PyTorch's caching allocator; the paper's method is unaffected).
 * By default the library takes its device buffers from hipMalloc.  After this
 * call, alloc(bytes, user) supplies every device buffer the library allocates
 * -- sim pools, task lists, flux registers, network weights and work arrays
 * -- and release(ptr, user) takes it back; both NULL restore hipMalloc /
 * hipFree.  alloc must return memory of the current device aligned to at
 * least 256 bytes, or NULL (the allocating call then fails with IC_E_NOMEM).
 * Every buffer goes back through the allocator it came from, also after a
 * later change.  Pinned host memory and the static scratch of
 * ic_mlp_infer_noalloc are not affected.  Process-wide: do not call it while
 * another thread is inside the library.  IC_E_INVALID if exactly one of alloc
 * and release is NULL. */
typedef void *(*ic_alloc_fn)(size_t bytes, void *user);
typedef void (*ic_free_fn)(void *ptr, void *user);
ic_status ic_set_device_allocator(ic_alloc_fn alloc, ic_free_fn release, void *user);

/* 1 if the library has kernels for this block shape, else 0. */
int ic_block_supported(int bi, int bj, int bk);

/* Kernel timing for measurement: when enabled, ic_step launches its kernels
 * without graph replay and brackets every launch of the finite-volume stage
 * kernel with HIP events on the sim's stream; ic_stage_timing returns the
 * number of timed launches and their mean duration [ms] since the last
 * reset (it synchronises the stream). */
ic_status ic_set_kernel_timing(ic_sim *sim, int enable);
ic_status ic_stage_timing(ic_sim *sim, long *launches, double *mean_ms);

/* Text of the last error on the calling thread. */
const char *ic_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ICARUS_H */
