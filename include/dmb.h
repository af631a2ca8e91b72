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
    DMB_RATES_QUAD = 1    /* K-node Gauss-Legendre quadrature of the radial form of eq. scrA/scrB */
} dmb_rates;

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
    double sigma0_cm2;      /* sigma(v) = sigma0 (v/c)^n, isotropic (Sec. 2.4) */
    int32_t n_pow;          /* n in {-4, -2, 0, 2} */
    double m_chi_g;         /* DM particle mass m_chi, g */
    double dt;              /* default timestep, kpc/(km/s) */
    uint64_t seed;          /* Philox key */
    uint32_t step;          /* step counter (Philox counter word 2) */
    uint32_t box_id;        /* box index (Philox counter word 3 bits 8..31) */
    double box[3];          /* periodic side lengths in kpc; all 0 => open boundaries */
    int32_t precision;      /* dmb_precision */
    int32_t rates;          /* dmb_rates */
    int32_t quad_nodes;     /* K for DMB_RATES_QUAD, 4..64; 0 => 32 */
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
 * direction is isotropic (tag 1) and dv_dm follows eq. scatter_chi.
 * Overlap g: exact (piecewise Gauss-Legendre) in DMB_FP64, table in DMB_FP32.
 * Errors: DMB_EINVAL, DMB_ESTALE. */
dmb_status dmb_interact_step(dmb_ctx *ctx, const dmb_particles *gas, const dmb_particles *dm,
                             const dmb_params *params, dmb_out *out);

/* Device-side evaluation helpers (synchronous; device arrays of length n).
 * dmb_overlap_eval: g(d; h1, h2) of eq. dm-update-prob / Appendix D, table
 *   (DMB_FP32) or exact (DMB_FP64).
 * dmb_rates_eval: A/(sigma0 c^-n), B/(sigma0 c^-n) of eq. scrA/scrB at speeds
 *   w and dispersions vs for power n, by the closed forms of Appendix B
 *   (rates = DMB_RATES_EXACT) or by quad_nodes-point quadrature (DMB_RATES_QUAD).
 * dmb_philox_eval: Philox4x32-10 blocks for counters ctr[n][4] under key
 *   (seed lo, seed hi), written to out[n][4]. */
dmb_status dmb_overlap_eval(dmb_ctx *ctx, int64_t n, const double *d, const double *h1, const double *h2,
                            int32_t precision, double *g_out);
dmb_status dmb_rates_eval(dmb_ctx *ctx, int64_t n, const double *w, const double *vs, int32_t n_pow,
                          int32_t precision, int32_t rates, int32_t quad_nodes, double *A_out, double *B_out);
dmb_status dmb_philox_eval(dmb_ctx *ctx, int64_t n, const uint32_t *ctr, uint64_t seed, uint32_t *out);

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

/* Structure of the last dmb_build_cells (host array of 10 int64):
 * [active gas, active DM, gas tiles, DM tiles, gas owner tiles, DM owner
 *  tiles, candidate tile pairs of the gas pass, of the DM pass, work items of
 *  the gas pass, of the DM pass]. */
dmb_status dmb_build_stats(const dmb_ctx *ctx, int64_t *out10);

/* Message for the last failure on this context; with ctx == NULL, the
 * message of the last failed dmb_create (never NULL). */
const char *dmb_last_error(const dmb_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* DMB_H */
