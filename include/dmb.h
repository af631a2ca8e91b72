/*
 * dmb.h -- C ABI of the MI355X (gfx950) DM-gas pair interaction library.
 *
 * Implements the per-step DM-baryon interaction of Hainje & Farrar, "A New
 * Method to Simulate Dark Matter-Baryon Interactions and Application to an
 * Isolated Disk Galaxy" (arXiv 2603.24688), Sec. 2:
 *   - gas particles receive the mean-field momentum and internal-energy
 *     transfer of eq. gas-dVdt / gas-dTdt (Appendix B);
 *   - each DM particle receives one Monte Carlo draw from the velocity mixture
 *     of eq. dm-update-vels with pair probabilities P_ij of eq. dm-update-prob,
 *     and the elastic kick of eq. scatter_chi off its sampled gas partner.
 *
 * Conventions for every entry point:
 *   - Array pointers are DEVICE pointers owned by the caller; the library never
 *     frees or retains them beyond the call (build_cells keeps a sorted copy).
 *   - Work is enqueued on the context's stream; calls return without waiting
 *     for the GPU, except dmb_build_cells, which reads two counts back to size
 *     its buffers, and the *_eval helpers, which are synchronous.
 *   - Return value: DMB_OK (0) or a negative dmb_status.  On error nothing has
 *     been enqueued and dmb_last_error() describes the failure.
 *   - Units: kpc, km/s, Msun; times in kpc/(km/s); sigma0 in cm^2; m_chi and
 *     mu in grams; gas specific internal energy u in (km/s)^2 with 1-D velocity
 *     variance varsigma^2 = T/mu = 2u/3.
 *   - Indices: particle k of an array is identified by its index k; random
 *     numbers are keyed by (DM index, gas index, step, tag, box id), so results
 *     do not depend on ordering, tiling or launch shape.
 *   - One context per stream; a context is not thread-safe.
 */
#ifndef DMB_H
#define DMB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dmb_ctx dmb_ctx;

typedef enum {
    DMB_OK = 0,
    DMB_EINVAL = -1,      /* bad argument (null pointer, n < 0, unsupported option) */
    DMB_ENOMEM = -2,      /* device allocation failed */
    DMB_EHIP = -3,        /* HIP runtime error */
    DMB_ERANGE = -4,      /* h_i + h_j >= L/2 in a periodic box, or n >= 2^31 */
    DMB_ESTALE = -5       /* interact_step without a matching build_cells */
} dmb_status;

typedef enum { DMB_FP64 = 0, DMB_FP32 = 1 } dmb_precision;

/* How the rate integrals A, B (eq. scrA, scrB) are evaluated in the gas pass. */
typedef enum {
    DMB_RATES_EXACT = 0,  /* closed forms of the 1F1 expressions of Appendix B (integer n) */
    DMB_RATES_QUAD = 1,   /* K-node Gauss-Legendre quadrature of the radial form of eq. scrA/scrB */
    DMB_RATES_MLP = 2,    /* learned closure (dmb_mlp_*), binary32 only; K-node quadrature where the
                             similarity variable u = w/varsigma exceeds the trained range (u > 1000) */
    DMB_RATES_CLOSURE = 3 /* per-gas Maxwellian closure (the Appendix F rates applied per gas particle):
                             the gas pass sums the kernel-weighted DM density, drift and dispersion
                             around each gas particle (binary64 sums in either precision) and the
                             closed-form rates are evaluated once per gas particle at the combined
                             dispersion.  Exact for Maxwellian DM; the DM Monte Carlo is unchanged.
                             Not for dmb_rates_eval. */
} dmb_rates;

/* DM Monte Carlo sampling (Sec. 2.2 and an exact-in-law variant). */
typedef enum {
    DMB_SAMPLE_PAIR = 0,  /* the paper's scheme: one Maxwellian gas-velocity sample v_B per pair (Philox
                             tag 0), P_ij = K_j g_ij sigma(|v_i - v_B|) |v_i - v_B| dt_i */
    DMB_SAMPLE_RB = 1     /* Rao-Blackwellised: P_ij replaced by its expectation over v_B (the B rate
                             integral of power n - 2), and only a DM that scatters draws the relative
                             velocity of its chosen pair, from the |u|^{n+1}-tilted Maxwellian (Philox
                             tag 5, by inversion).  The same joint law of partner and kick as
                             DMB_SAMPLE_PAIR while P_i <= 1, with no per-pair random numbers.
                             n_pow > -4 only (the expectation diverges at n = -4): DMB_EINVAL. */
} dmb_dm_sampling;

enum {
    DMB_C_PAIRS_GAS = 0,  /* pairs visited by the gas (mean-field) pass */
    DMB_C_PAIRS_DM,       /* pairs visited by the DM (Monte Carlo) pass */
    DMB_C_SCATTERS,       /* DM particles that scattered */
    DMB_C_NEAR_BOUNDARY,  /* DM with a pair at |d^2/(h_i+h_j)^2 - 1| <= 1e-6 */
    DMB_C_NEAR_DECISION,  /* DM whose uniform lies within 1e-6 (relative) of a running sum */
    DMB_C_CRIT_VIOL,      /* pairs with P_ij >= min(0.1, 1e-4 ((m_chi+mu)/mu)^2), eq. prob_criterion */
    DMB_C_P_GE_1,         /* DM with sum_j P_ij >= 1 (always scatter) */
    DMB_C_NONFINITE,      /* DM with a non-finite P_ij */
    DMB_NCOUNTERS
};

/* One particle species (Sec. 2.1: macroparticle DFs eq. macroparticle-DF_DM /
 * macroparticle-DF_B).  All arrays are device arrays of length n (x3 for
 * vectors, row-major [n][3]). */
typedef struct {
    int64_t n;
    const double *pos;      /* [n][3] position, kpc */
    const double *vel;      /* [n][3] velocity (gas: bulk velocity V_j), km/s */
    const double *mass;     /* [n] macroparticle mass M, Msun */
    const double *h;        /* [n] kernel support radius h (W = 0 for r >= h), kpc */
    const double *u;        /* gas: [n] specific internal energy, (km/s)^2; DM: NULL */
    const double *mu;       /* gas: [n] mean molecular weight, g; NULL => proton mass */
    const uint8_t *active;  /* [n] nonzero = active this step; NULL => all active */
    const double *dt;       /* [n] per-particle timestep; NULL => params.dt */
} dmb_particles;

typedef struct {
    double sigma0_cm2;      /* total cross section sigma(v) = sigma0 (v/c)^n (Sec. 2.4) */
    int32_t n_pow;          /* n in {-4, -2, 0, 2} */
    double m_chi_g;         /* DM particle mass m_chi, g */
    double dt;              /* default timestep, kpc/(km/s) */
    uint64_t seed;          /* Philox key */
    uint32_t step;          /* step counter (Philox counter word 2) */
    uint32_t box_id;        /* box index (Philox counter word 3 bits 8..31) */
    double box[3];          /* periodic side lengths in kpc; all 0 => open boundaries */
    int32_t precision;      /* dmb_precision */
    int32_t rates;          /* dmb_rates */
    int32_t quad_nodes;     /* K for DMB_RATES_QUAD (and the DMB_RATES_MLP fallback), 4..64; 0 => 32.
                               K >= 24 integrates over w/vs +- 8.5, smaller K over +- 5.5 */
    double aniso_g;         /* angular shape of dsigma/dOmega = sigma(v) p(Omega) (Sec. 2.2-2.3): the
                               Henyey-Greenstein law in the scattering angle theta of the relative
                               velocity, mean cos theta = g, |g| < 1; 0 => isotropic.  The DM Monte
                               Carlo uses sigma and draws theta from p; the gas mean field uses the
                               momentum-transfer cross section sigma-bar = (1 - g) sigma (eq. scrA,
                               scrB).  Errors: DMB_EINVAL unless |g| < 1. */
    int32_t dm_sampling;    /* dmb_dm_sampling: how the DM Monte Carlo handles the gas-velocity sample */
} dmb_params;

typedef struct {
    double *dv_dm;          /* [n_dm][3] velocity change of each DM particle, km/s */
    double *dp_gas;         /* [n_gas][3] momentum change M_j dV_j, Msun km/s */
    double *de_gas;         /* [n_gas] internal-energy change M_j du_j, Msun (km/s)^2;
                               the bulk-kinetic part is V_j . dp_gas (Appendix C) */
    int32_t *partner;       /* [n_dm] scattering partner (gas index) or -1 */
    double *p_sum;          /* [n_dm] sum_j P_ij (nullable) */
    double *p_max;          /* [n_dm] max_j P_ij (nullable) */
    uint64_t *counters;     /* [DMB_NCOUNTERS] device, nullable; overwritten by the call */
} dmb_out;

/* Create a context on HIP device `device` that enqueues on `hip_stream`
 * (a hipStream_t, NULL = default stream).  Builds the overlap table on the
 * device.  *ctx receives the context; release it with dmb_destroy. */
dmb_status dmb_create(dmb_ctx **ctx, int device, void *hip_stream);
dmb_status dmb_destroy(dmb_ctx *ctx);
dmb_status dmb_set_stream(dmb_ctx *ctx, void *hip_stream);

/* Neighbour structure (Sec. 2.4: each overlapping pair d_ij < h_i + h_j is
 * processed once; Appendix D: the overlap vanishes beyond h_i + h_j).
 * Morton-sorts both species, forms 64-particle tiles and 4096-particle
 * super-tiles with bounding boxes and h_max, and lists, for every tile of
 * active owners, the tiles of the other species that can overlap it.
 * Captures pos, h and active of both species; call again whenever they
 * change.  Synchronises the stream once (to size the candidate lists).
 * Errors: DMB_EINVAL (null pos/h, n < 0), DMB_ERANGE (periodic box with
 * max h_gas + max h_dm >= L/2), DMB_ENOMEM. */
dmb_status dmb_build_cells(dmb_ctx *ctx, const dmb_particles *gas, const dmb_particles *dm,
                           const dmb_params *params);

/* One interaction step (Sec. 2.2-2.4) with the structure of the last
 * dmb_build_cells (same n, pos, h, active).  Reads vel, mass, u, mu, dt.
 * Gas pass: for every active gas j, sums over all overlapping DM i the terms
 * of eq. gas-dVdt / gas-dTdt (A, B of Appendix B) in double.  DM pass: for
 * every active DM i, P_ij = (M_j/mu_j) g_ij sigma(v_rel) v_rel dt_i with one
 * Maxwellian gas-velocity sample per pair (Philox tag 0); one uniform U_i
 * (tag 2) decides a scatter if U_i < sum_j P_ij; the partner is the first gas
 * index (ascending) whose running sum exceeds U_i; the new relative-velocity
 * direction is isotropic (tag 1, or Henyey-Greenstein about the incoming
 * direction when aniso_g != 0) and dv_dm follows eq. scatter_chi.
 * Overlap g: exact (piecewise Gauss-Legendre) in DMB_FP64, table in DMB_FP32.
 * DMB_FP32 forms the pair terms in binary32 and sums them in binary64; the
 * kick of a scattering DM (its pair's sample and dv_dm) is binary64 in
 * either precision.
 * Errors: DMB_EINVAL, DMB_ESTALE. */
dmb_status dmb_interact_step(dmb_ctx *ctx, const dmb_particles *gas, const dmb_particles *dm,
                             const dmb_params *params, dmb_out *out);

/* ------------------------------------------------------------------------
 * Time loop.  nsteps steps of the method on one volume: each step rebuilds
 * the neighbour structure, runs dmb_interact_step, then applies the DM kicks
 * and the gas momentum and internal-energy transfers (from start-of-step
 * states) and drifts both species with their new velocities (wrapped into
 * [0, L) when periodic).  gas->pos, gas->vel, gas->u, dm->pos and dm->vel are
 * UPDATED IN PLACE (device arrays).  Step k uses Philox step params->step + k.
 * Timestep control (eq. prob_criterion, applied to the next step as the
 * paper's implementation does): with cfg->dt_control, step k+1 takes
 * dt = min(dt_max, dt_k * safety * crit / max_ij P_ij) where crit is the
 * smallest criterion min(0.1, 1e-4 ((m_chi + mu_j)/mu_j)^2) over the gas;
 * otherwise every step takes dt_max.  A per-particle dt is not allowed here.
 * diag (HOST, (nsteps + 1) x DMB_NDIAG doubles): row 0 the initial state, row
 * k the state after step k; all sums in binary64 in a fixed order. */
enum {
    DMB_D_TIME = 0,                 /* elapsed time, kpc/(km/s) */
    DMB_D_DT = 1,                   /* length of this step (0 in row 0) */
    DMB_D_P_DM = 2,                 /* [3] total DM momentum sum M v, Msun km/s */
    DMB_D_P_GAS = 5,                /* [3] total gas momentum sum M V */
    DMB_D_E_DM = 8,                 /* DM kinetic energy sum M v^2/2, Msun (km/s)^2 */
    DMB_D_E_GAS = 9,                /* gas energy sum M (V^2/2 + u) (bulk kinetic + internal) */
    DMB_D_V_DM = 10,                /* [3] mass-weighted mean DM velocity, km/s */
    DMB_D_V_GAS = 13,               /* [3] mass-weighted mean gas velocity */
    DMB_D_S2_DM = 16,               /* DM 1-D velocity variance about the mean (T_DM = m_chi s2), (km/s)^2 */
    DMB_D_S2_GAS = 17,              /* gas 1-D variance: 2<u>/3 + <|V - <V>|^2>/3 (T_gas = mu s2) */
    DMB_D_JB_DM = 18,               /* largest Jarque-Bera statistic (S^2 + (K-3)^2/4)/6 of the three DM
                                       velocity components, without the sample-size factor (Appendix F) */
    DMB_D_SCATTERS = 19,            /* DM that scattered in the step */
    DMB_D_CRIT_VIOL = 20,           /* pairs above the criterion of eq. prob_criterion in the step */
    DMB_D_P_MAX = 21,               /* largest P_ij of the step */
    DMB_D_PAIRS = 22,               /* pairs visited by the DM pass in the step (active DM) */
    DMB_D_PAIRS_GAS = 23,           /* pairs visited by the gas pass in the step (active gas) */
    DMB_NDIAG = 24
};
typedef struct {
    int32_t nsteps;                 /* >= 0 */
    int32_t dt_control;             /* nonzero: limit dt by the scattering-probability criterion */
    double dt_max;                  /* nominal (and largest) step, kpc/(km/s) */
    double safety;                  /* fraction of the criterion aimed at, in (0, 1] */
    double active_frac;             /* 0: the particles' own active arrays every step; in (0, 1]: each step k
                                       draws the active set of each species afresh (hierarchical timesteps):
                                       particle i of species s (0 gas, 1 DM) is active iff the first word r0
                                       of Philox4x32-10 (key = seed, counter = (i, s, step + k, 3 | box << 8))
                                       gives ((r0 >> 8) + 1/2) 2^-24 < active_frac */
} dmb_run_cfg;
/* Errors: those of dmb_build_cells / dmb_interact_step; DMB_EINVAL for a null
 * cfg or diag, nsteps < 0, dt_max <= 0, safety outside (0, 1], active_frac
 * outside [0, 1], or per-particle dt arrays. */
dmb_status dmb_run(dmb_ctx *ctx, const dmb_particles *gas, const dmb_particles *dm, const dmb_params *params,
                   const dmb_run_cfg *cfg, double *diag);

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): dmb_build_cells
 * followed by dmb_interact_step in one call, with every scratch buffer of
 * both carved from a static device array of DMB_STATIC_SCRATCH_MIB MiB
 * instead of device allocations.  Each GPU the library runs on holds its own
 * copy of the array until the process ends (looked up by dmb_create).
 * The caller passes inputs and outputs as for dmb_interact_step, and the
 * outputs are identical to theirs.  Limits: n_gas, n_dm <= DMB_STATIC_MAX_N;
 * rates DMB_RATES_EXACT; phase timing off.  Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (from any context or
 * stream) race; the array keeps the last call's contents and every call
 * rebuilds what it reads.  The structure of the last dmb_build_cells on ctx is
 * left untouched.  Synchronises the stream (as dmb_build_cells does).
 * Errors: those of dmb_build_cells / dmb_interact_step; DMB_ERANGE for sizes
 * above the limit; DMB_EINVAL for other rate modes or with phase timing on;
 * DMB_ENOMEM when the inputs need more scratch than the array holds (very
 * dense neighbour structures). */
#define DMB_STATIC_SCRATCH_MIB 256
#define DMB_STATIC_MAX_N 262144
dmb_status dmb_step_static(dmb_ctx *ctx, const dmb_particles *gas, const dmb_particles *dm,
                           const dmb_params *params, dmb_out *out);

/* The pair set of Sec. 2.4 (every overlapping pair d_ij < h_i + h_j, the
 * support of the overlap of Appendix D, processed once per pass) as the two
 * pair passes enumerate it.  Runs one interaction step exactly as
 * dmb_interact_step (same outputs in *out) and also writes each pair that the
 * gas pass and the DM pass visit, as (DM index, gas index) uint32 pairs, into
 * pairs_gas[cap][2] and pairs_dm[cap][2] (device, caller-owned), in no
 * particular order.  counts (HOST, 2 int64) receives each pass's total; when
 * a total exceeds cap, only cap pairs of that pass are written.  For checking
 * the neighbour structure: the step must use n_pow = 0, DMB_RATES_EXACT
 * and DMB_SAMPLE_PAIR (the pair set depends on none of them).  Synchronous.
 * Errors: those of dmb_interact_step; DMB_EINVAL for n_pow != 0, other rate
 * or sampling modes, cap < 0, or null lists with cap > 0. */
dmb_status dmb_pair_list(dmb_ctx *ctx, const dmb_particles *gas, const dmb_particles *dm,
                         const dmb_params *params, dmb_out *out, int64_t cap, uint32_t *pairs_gas,
                         uint32_t *pairs_dm, int64_t *counts);

/* The stable radix sort that orders particles along the Morton curve for the
 * neighbour search (Sec. 2.4) and work items by size: sorts n (key, value)
 * pairs by the key bits [lo_bit, lo_bit + 8 passes), ties kept in input
 * order.  keys_in/vals_in, keys_out/vals_out: device arrays of n (the
 * inputs are not modified; outputs must not alias them).  Synchronous.
 * Errors: DMB_EINVAL (n < 0 or >= 2^31, null arrays, passes outside 1..8,
 * bits outside the key), DMB_ENOMEM, DMB_EHIP. */
dmb_status dmb_sort_pairs(dmb_ctx *ctx, int64_t n, const uint64_t *keys_in, const uint32_t *vals_in, int32_t lo_bit,
                          int32_t passes, uint64_t *keys_out, uint32_t *vals_out);

/* Device-side evaluation helpers (synchronous; device arrays of length n).
 * dmb_overlap_eval: g(d; h1, h2) of eq. dm-update-prob / Appendix D, table
 *   (DMB_FP32: relative error below 1e-6 everywhere inside the support) or
 *   exact (DMB_FP64).
 * dmb_rates_eval: A/(sigma0 c^-n), B/(sigma0 c^-n) of eq. scrA/scrB at speeds
 *   w and dispersions vs for power n, by the closed forms of Appendix B
 *   (rates = DMB_RATES_EXACT), by quad_nodes-point quadrature (DMB_RATES_QUAD)
 *   or by the loaded network (DMB_RATES_MLP, binary32 whatever precision says,
 *   with the arithmetic of the interaction step).
 * dmb_philox_eval: Philox4x32-10 blocks for counters ctr[n][4] under key
 *   (seed lo, seed hi), written to out[n][4]. */
dmb_status dmb_overlap_eval(dmb_ctx *ctx, int64_t n, const double *d, const double *h1, const double *h2,
                            int32_t precision, double *g_out);
dmb_status dmb_rates_eval(dmb_ctx *ctx, int64_t n, const double *w, const double *vs, int32_t n_pow,
                          int32_t precision, int32_t rates, int32_t quad_nodes, double *A_out, double *B_out);
dmb_status dmb_philox_eval(dmb_ctx *ctx, int64_t n, const uint32_t *ctr, uint64_t seed, uint32_t *out);

/* ------------------------------------------------------------------------
 * Batched boxes: parameter sweeps over many independent volumes (each with
 * its own sigma0, m_chi, periodic box, particle counts) run as one step.
 * Each box keeps its own Morton cell structure; each of the two pair passes
 * is one persistent launch over the work items of all boxes.  gas, dm, par
 * and out are HOST arrays of nbox structs pointing at device data; every
 * box's out.counters must be set.  n_pow, precision, rates and quad_nodes
 * must agree across boxes.  Results per box are those of dmb_build_cells +
 * dmb_interact_step on that box with the same tuning.
 */
/* Cell structures of all boxes (as dmb_build_cells, box by box).
 * Errors: as dmb_build_cells, the message naming the box. */
dmb_status dmb_batch_build(dmb_ctx *ctx, int32_t nbox, const dmb_particles *gas, const dmb_particles *dm,
                           const dmb_params *par);
/* nsteps interaction steps of every box; step k uses Philox step
 * par[b].step + k; outputs hold the last step.  use_graph != 0 captures one
 * step as a hipGraph (on the context stream, or on a private non-blocking
 * stream when the context uses the default stream) and replays it nsteps
 * times; the call then waits for the GPU.  Errors: DMB_EINVAL, DMB_ESTALE
 * (sizes differ from the last dmb_batch_build), DMB_EHIP. */
dmb_status dmb_batch_step(dmb_ctx *ctx, int32_t nbox, const dmb_particles *gas, const dmb_particles *dm,
                          const dmb_params *par, dmb_out *out, int32_t nsteps, int32_t use_graph);
/* Autotuner: times the batched step over work-item sizes {32, 64, 128}
 * candidate sub-tiles, sub-tile granularities (cut at Morton level median -
 * {0, 1, 2}) and persistent grids of {50, 100} % of the resident maximum,
 * keeps the fastest setting in the context (it applies to every later build
 * and step) and rebuilds the boxes with it.  choice (HOST, 4 int64, nullable)
 * receives {work-item size, granularity, grid %, microseconds per step}.
 * Overwrites the outputs.  Errors: as dmb_batch_step. */
dmb_status dmb_batch_tune(dmb_ctx *ctx, int32_t nbox, const dmb_particles *gas, const dmb_particles *dm,
                          const dmb_params *par, dmb_out *out, int64_t *choice);

/* ------------------------------------------------------------------------
 * Learned closure for the rate integrals (an extension of the method: the
 * paper evaluates eq. scrA / scrB through 1F1; here a small network may stand
 * in for them, with quadrature as its judge and fallback).
 *
 * Inputs per sample, x[k][4] (device, binary64): x1 = w / varsigma_gas,
 * x2 = T_DM / T_gas, x3 = log10(m_chi / mu), x4 = n in {-4, -2, 0, 2}.
 * A Maxwellian DM population makes the relative velocity Gaussian with
 * dispersion vth = varsigma_gas r, r = sqrt(1 + x2 10^{-x3}) (x2 = 0 in the
 * interaction step, where each DM particle has one velocity), so with
 * u = x1 / r (Appendix B):
 *   Ahat / vs^{n+1} = r^{n+1} (alpha_n/3) 1F1(-(n+1)/2, 5/2, -u^2/2),
 *   Bhat / vs^{n+3} = r^{n+3}  alpha_n    1F1(-(n+3)/2, 3/2, -u^2/2).
 * The network (inputs s = 2u/(u+2) - 1 and one-hot n; three 64-unit ReLU
 * layers; two outputs) predicts y = (ln of the two 1F1 terms) minus
 * (ln a_A(u), ln a_B(u)), a = (c0 + c1 u^2 + u^4)^{p/4} with p = n+1 (A),
 * n+3 (B), c0 = (u = 0 value)^{4/p} (values alpha_n/3 and alpha_n), and
 * c1 = (0.833, 0.694), (4.327, 4.114), (8.061, 7.967), (11.981, 12.089) for
 * n = -4, -2, 0, 2 (A, B).  bfloat16 weights and
 * activations, binary32 accumulation (MFMA); binary32 master weights.
 * Parameter vector (binary32, DMB_MLP_PARAMS values, row-major W[out][in]):
 *   W1[64][5] b1[64] W2[64][64] b2[64] W3[64][64] b3[64] W4[2][64] b4[2].
 * The context owns the weights; all calls below are synchronous.
 */
#define DMB_MLP_PARAMS 8834

typedef struct {
    int32_t epochs;         /* passes over the training set */
    int32_t batch;          /* samples per Adam step: a positive multiple of 64, <= n */
    double lr0, lr_min;     /* cosine learning rate from lr0 (first step) towards lr_min */
    double beta1, beta2, eps;  /* Adam (Kingma & Ba 2015) */
    uint64_t seed;          /* epoch shuffles; and the initial weights when init != 0 */
    int32_t init;           /* nonzero: draw fresh He-uniform weights from seed first */
    int32_t use_graph;      /* nonzero: capture one epoch as a hipGraph and replay it */
} dmb_mlp_train_cfg;

/* Residual targets y[n][2] (device, binary64) for inputs x[n][4] by
 * quad_nodes-point (0 => 48) binary64 quadrature of the rate integrals.
 * Errors: DMB_EINVAL (bad pointers, n < 0, quad_nodes outside 4..64). */
dmb_status dmb_mlp_labels(dmb_ctx *ctx, int64_t n, const double *x, int32_t quad_nodes, double *y);
/* Fresh weights from Philox (counter = (parameter, 0, 0, 4), key = seed). */
dmb_status dmb_mlp_init(dmb_ctx *ctx, uint64_t seed);
/* Copy the parameter vector from / to HOST memory (count == DMB_MLP_PARAMS). */
dmb_status dmb_mlp_set_params(dmb_ctx *ctx, const float *params, int64_t count);
dmb_status dmb_mlp_get_params(dmb_ctx *ctx, float *params, int64_t count);
/* Loss L = 100 sum_{k,o} (out_ko - y_ko)^2 / (2n) over the n samples as one
 * batch and its gradient (straight-through bfloat16 rounding) with respect to
 * the parameters.  x, y device; grad a HOST array of DMB_MLP_PARAMS floats;
 * loss a HOST double (nullable).  Errors: DMB_EINVAL (n < 1, no weights). */
dmb_status dmb_mlp_grad(dmb_ctx *ctx, int64_t n, const double *x, const double *y, float *grad, double *loss);
/* Train on n samples (x, y device) with Adam: epochs x floor(n / batch)
 * steps; forward and backward on MFMA.  epoch_loss: HOST array of cfg->epochs
 * mean training losses (nullable).  Errors: DMB_EINVAL, DMB_EHIP. */
dmb_status dmb_mlp_train(dmb_ctx *ctx, int64_t n, const double *x, const double *y, const dmb_mlp_train_cfg *cfg,
                         double *epoch_loss);
/* Network estimate of (ln Ahat/vs^{n+1}, ln Bhat/vs^{n+3}) into out[n][2]
 * (device, binary64); u > 1000 by binary64 quadrature.  Errors: DMB_EINVAL. */
dmb_status dmb_mlp_eval(dmb_ctx *ctx, int64_t n, const double *x, double *out);

/* Phase timing with HIP events recorded on the context stream around each
 * kernel group of dmb_build_cells / dmb_interact_step. */
enum {
    DMB_PH_BUILD = 0,     /* dmb_build_cells (whole call, including its read-back) */
    DMB_PH_GATHER,        /* per-step gathers into Morton order and output clears */
    DMB_PH_PASS_GAS,      /* gas mean-field pair pass */
    DMB_PH_COMBINE_GAS,   /* gas partial combine and output write */
    DMB_PH_PASS_DM,       /* DM Monte Carlo pair pass */
    DMB_PH_COMBINE_DM,    /* DM partial combine and scatter decision */
    DMB_PH_RESOLVE,       /* partner resolve and kick of scattering DM */
    DMB_NPHASES
};
/* on != 0 starts recording (costs two event records per phase). */
dmb_status dmb_profile_enable(dmb_ctx *ctx, int32_t on);
/* Waits for recorded work, then writes accumulated milliseconds and call
 * counts per phase (host arrays of DMB_NPHASES); reset != 0 clears them. */
dmb_status dmb_profile_read(dmb_ctx *ctx, double *ms, int64_t *calls, int32_t reset);

/* Candidate-search groups (a tuning control of the neighbour structure that
 * dmb_build_cells forms for Sec. 2.4's pairs d_ij < h_i + h_j: which
 * other-species super-tiles each owner tile of 64 owners may reach).
 * Outputs never depend on it.  A first pass lists the candidates of each group of
 * 64 consecutive owner tiles, keeping up to `cap` of them; each tile whose
 * group list fits tests only that list, the others walk the full node
 * hierarchy.  Both give the same candidate lists in the same order.
 * cap = 0 turns the group pass off; default 1024.
 * Applies to later dmb_build_cells / dmb_batch_build calls.  Errors:
 * DMB_EINVAL for a null ctx or cap outside [0, 65536]. */
dmb_status dmb_set_search_groups(dmb_ctx *ctx, int32_t cap);

/* Pass overlap (a scheduling control of dmb_interact_step; outputs never
 * depend on it).  on = 1 (default): the gas pass and its combine run on an
 * internal stream while the DM pass, its decisions and the resolve run on the
 * context's stream, so both persistent passes share the GPU.  on = 0: one
 * after the other on the context's stream, so that phase timing
 * (dmb_profile_read) gives each pass's own time.  The batched step follows the
 * same setting (its two streams are forked and joined inside the captured
 * graph when it replays).  Errors: DMB_EINVAL for a null ctx. */
dmb_status dmb_set_pass_overlap(dmb_ctx *ctx, int32_t on);

/* Structure of the last dmb_build_cells (host array of 10 int64):
 * [active gas, active DM, gas tiles, DM tiles, gas owner tiles, DM owner
 *  tiles, candidate (owner tile, sub-tile) pairs of the gas pass, of the DM
 *  pass, work items of the gas pass, of the DM pass]. */
dmb_status dmb_build_stats(const dmb_ctx *ctx, int64_t *out10);

/* Message for the last failure on this context; with ctx == NULL, the
 * message of the last failed dmb_create (never NULL). */
const char *dmb_last_error(const dmb_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DMB_H */
