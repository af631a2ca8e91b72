/*
 * dmb_oracle.c -- plain, slow FP64 CPU oracle for the DM-gas pair interaction
 * step of Hainje & Farrar, "A New Method to Simulate Dark Matter-Baryon
 * Interactions and Application to an Isolated Disk Galaxy" (arXiv 2603.24688).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code, header, table or constant with
 * the HIP path.
 *
 * Everything is IEEE double.  Neighbours are found by brute force, or, for
 * large inputs, among the candidates of a set of uniform grids (orc_grid_*):
 * every candidate still passes the same pair test and sums run in the same
 * ascending index order, so both give bit-identical results.  Each function
 * cites the passage of the paper it writes out.
 *
 * Units: kpc, km/s, Msun; time in kpc/(km/s); sigma0 in cm^2; m_chi, mu in g;
 * gas specific internal energy u in (km/s)^2, 1-D velocity variance
 * varsigma^2 = 2u/3 (= T/mu with k_B absorbed).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define ORC_PI 3.14159265358979323846
#define ORC_MSUN_G 1.988409870698051e33
#define ORC_KPC_CM 3.0856775814913673e21
#define ORC_C_KMS 299792.458
#define ORC_MP_G 1.67262192369e-24

/* ------------------------------------------------------------------------- */
/* Cubic-spline softening kernel (Sec. 2.4, "GIZMO implementation"):
 * W(r,h) = w(r/h)/h^3 with w(q) = 8/pi * {1-6q^2+6q^3, q<=1/2; 2(1-q)^3,
 * 1/2<q<=1; 0, q>1}.                                                        */
double orc_w(double q)
{
    if (q < 0.0) q = -q;
    if (q <= 0.5) return (8.0 / ORC_PI) * (1.0 - 6.0 * q * q + 6.0 * q * q * q);
    if (q <= 1.0) { double p = 1.0 - q; return (8.0 / ORC_PI) * 2.0 * p * p * p; }
    return 0.0;
}

double orc_W(double r, double h) { return orc_w(r / h) / (h * h * h); }

/* ------------------------------------------------------------------------- */
/* Overlap integral g_ij (eq. dm-update-prob; Appendix D).
 *
 * g = int d^3x W(|x-x_i|,h_i) W(|x-x_j|,h_j).  Appendix D reduces it, with
 * the outer radial integral over the kernel with the larger h (h_b) and the
 * ratio eta = h_s/h_b <= 1, delta = d/h_b, to
 *     g = (2 pi / h_s^3) int_0^1 ds s^2 w(s) F(s),
 *     F(s) = int_{-1}^{1} dc w( sqrt(s^2 + delta^2 - 2 delta s c) / eta ).
 * Substituting t = sqrt(s^2+delta^2-2 delta s c) gives
 *     F(s) = eta^2/(delta s) [psi((s+delta)/eta) - psi(|s-delta|/eta)],
 *     psi(Q) = int_0^Q q w(q) dq,
 * a piecewise polynomial.  The s-integrand is therefore a polynomial of
 * degree <= 9 between the breakpoints {1/2, delta, delta +- eta/2,
 * delta +- eta, eta/2 - delta, eta - delta}, so 6-point Gauss-Legendre on each
 * piece is exact up to rounding.  No table.                                  */

/* psi on each branch; branch 0: Q<=1/2, 1: 1/2<Q<=1, 2: Q>1.                */
static int psi_branch(double Q) { return Q <= 0.5 ? 0 : (Q <= 1.0 ? 1 : 2); }

/* psi(b) - psi(a) for a, b inside one branch, in a factored form that keeps
 * relative accuracy when b - a is small; bma = b - a supplied by the caller. */
static double psi_diff_same_branch(int br, double a, double b, double bma)
{
    const double c = 8.0 / ORC_PI;
    if (br == 0) {
        /* psi = c [Q^2/2 - 3 Q^4/2 + 6 Q^5/5] */
        double s1 = a + b;
        double s3 = (a * a + b * b) * s1;                  /* b^4-a^4 = (b-a) s3 */
        double s4 = b * b * b * b + b * b * b * a + b * b * a * a + b * a * a * a + a * a * a * a;
        return c * bma * (0.5 * s1 - 1.5 * s3 + 1.2 * s4);
    }
    if (br == 1) {
        /* psi = const + c [ -(1-Q)^4/2 + 2 (1-Q)^5/5 ];  with p = 1-Q,
         * p_a - p_b = b - a.                                                */
        double pa = 1.0 - a, pb = 1.0 - b;
        double t3 = (pa * pa + pb * pb) * (pa + pb);       /* pa^4-pb^4 = (pa-pb) t3 */
        double t4 = pa * pa * pa * pa + pa * pa * pa * pb + pa * pa * pb * pb + pa * pb * pb * pb + pb * pb * pb * pb;
        return c * bma * (0.5 * t3 - 0.4 * t4);
    }
    return 0.0;
}

/* psi at the branch edges: psi(1/2) = c*11/160, psi(1) = c*7/80.           */
static double psi_edge(int k) { return (8.0 / ORC_PI) * (k == 0 ? 11.0 / 160.0 : 7.0 / 80.0); }

/* psi(b) - psi(a), 0 <= a <= b, with bma = b - a given.                      */
static double psi_diff(double a, double b, double bma)
{
    int ba = psi_branch(a), bb = psi_branch(b);
    if (ba == bb) return psi_diff_same_branch(ba, a, b, bma);
    double acc = 0.0, lo = a;
    int br = ba;
    while (br < bb) {
        double edge = (br == 0) ? 0.5 : 1.0;
        acc += psi_diff_same_branch(br, lo, edge, edge - lo);
        lo = edge;
        br++;
    }
    acc += psi_diff_same_branch(bb, lo, b, b - lo);
    return acc;
}

static const double GL6_X[6] = {-0.9324695142031521, -0.6612093864662645, -0.2386191860831969,
                                 0.2386191860831969, 0.6612093864662645, 0.9324695142031521};
static const double GL6_W[6] = {0.1713244923791704, 0.3607615730481386, 0.4679139345726910,
                                 0.4679139345726910, 0.3607615730481386, 0.1713244923791704};

/* Integrand s^2 w(s) F(s) of Appendix D (without the 2 pi/h_s^3 prefactor). */
static double overlap_integrand(double s, double delta, double eta)
{
    double ws = orc_w(s);
    if (ws == 0.0) return 0.0;
    double F;
    if (delta == 0.0) {
        F = 2.0 * orc_w(s / eta);                       /* limit delta -> 0 */
    } else {
        double a = fabs(s - delta) / eta, b = (s + delta) / eta;
        double bma = 2.0 * (s < delta ? s : delta) / eta;
        F = eta * eta / (delta * s) * psi_diff(a, b, bma);
    }
    return s * s * ws * F;
}

static int cmp_double(const void *x, const void *y)
{
    double a = *(const double *)x, b = *(const double *)y;
    return (a > b) - (a < b);
}

/* Dimensionless G(delta, eta) = int_0^1 ds s^2 w(s) F(s); g = 2 pi G / h_s^3. */
double orc_overlap_G(double delta, double eta)
{
    if (delta >= 1.0 + eta) return 0.0;
    double bp[16];
    int nb = 0;
    double cand[9] = {0.0, 1.0, 0.5, delta, delta - 0.5 * eta, delta + 0.5 * eta,
                      delta - eta, delta + eta, 0.5 * eta - delta};
    for (int k = 0; k < 9; k++) {
        double v = cand[k];
        if (v >= 0.0 && v <= 1.0) bp[nb++] = v;
    }
    if (eta - delta > 0.0 && eta - delta < 1.0) bp[nb++] = eta - delta;
    qsort(bp, (size_t)nb, sizeof(double), cmp_double);
    double acc = 0.0;
    for (int k = 0; k + 1 < nb; k++) {
        double lo = bp[k], hi = bp[k + 1];
        if (hi <= lo) continue;
        double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo);
        double piece = 0.0;
        for (int q = 0; q < 6; q++) piece += GL6_W[q] * overlap_integrand(mid + half * GL6_X[q], delta, eta);
        acc += half * piece;
    }
    return acc;
}

double orc_overlap(double d, double h1, double h2)
{
    double hb = h1 > h2 ? h1 : h2, hs = h1 > h2 ? h2 : h1;
    double delta = d / hb, eta = hs / hb;
    return 2.0 * ORC_PI * orc_overlap_G(delta, eta) / (hs * hs * hs);
}

/* ------------------------------------------------------------------------- */
/* Confluent hypergeometric 1F1(a, b; -x), x >= 0 (Sec. 2.4 and Appendix B).
 * x < 50: Kummer's transformation 1F1(a,b;-x) = e^{-x} 1F1(b-a,b;x) and the
 * defining power series (all terms positive when b-a > 0 and b > 0).
 * x >= 50: the paper's expansion Gamma(b) x^{-a} / Gamma(b-a) *
 * sum_{k=0}^{4} (a)_k (1+a-b)_k / (k! x^k), truncated at five terms.         */
double orc_hyp1f1_negx(double a, double b, double x)
{
    if (x < 50.0) {
        double c = b - a, term = 1.0, sum = 1.0;
        for (int k = 0; k < 2000; k++) {
            term *= (c + k) / (b + k) * x / (k + 1.0);
            sum += term;
            if (term < 1e-18 * sum) break;
        }
        return exp(-x) * sum;
    }
    double pre = exp(lgamma(b) - lgamma(b - a)) * pow(x, -a);
    /* Gamma(b-a) may be negative for b-a<0; not reached for the (a,b) used here. */
    double term = 1.0, sum = 1.0;
    for (int k = 0; k < 4; k++) {
        term *= (a + k) * (1.0 + a - b + k) / ((k + 1.0) * x);
        sum += term;
    }
    return pre * sum;
}

/* orc_hyp1f1_negx over an array (labels for the learned closure).          */
void orc_hyp1f1_negx_v(long n, double a, double b, const double *x, double *out)
{
    for (long k = 0; k < n; k++) out[k] = orc_hyp1f1_negx(a, b, x[k]);
}

/* alpha_n = 2^{(n+5)/2} Gamma(3+n/2) / sqrt(pi)  (Appendix B).               */
double orc_alpha_n(int n) { return pow(2.0, 0.5 * (n + 5)) * tgamma(3.0 + 0.5 * n) / sqrt(ORC_PI); }

/* Rate integrals (eq. scrA, scrB) for sigma-bar = sigma0 (v/c)^n, written
 * without the factor sigma0 c^{-n}:
 *   Ahat = alpha_n/3 vs^{n+1} 1F1(-(n+1)/2, 5/2, -w^2/(2 vs^2)),
 *   Bhat = alpha_n   vs^{n+3} 1F1(-(n+3)/2, 3/2, -w^2/(2 vs^2)).
 * vs = varsigma (km/s), w = |w| (km/s).  vs = 0 (cold gas) takes the limit
 * Ahat = w^{n+1}, Bhat = w^{n+3}.                                            */
void orc_rates(int n, double w, double vs, double *A, double *B)
{
    if (vs <= 0.0) {
        *A = pow(w, n + 1);
        *B = pow(w, n + 3);
        return;
    }
    double x = w * w / (2.0 * vs * vs);
    double al = orc_alpha_n(n);
    *A = al / 3.0 * pow(vs, n + 1) * orc_hyp1f1_negx(-0.5 * (n + 1), 2.5, x);
    *B = al * pow(vs, n + 3) * orc_hyp1f1_negx(-0.5 * (n + 3), 1.5, x);
}

/* ------------------------------------------------------------------------- */
/* Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11,
 * "Parallel Random Numbers: As Easy as 1, 2, 3"), written from the published
 * description: each round takes the two 32x32->64 products of (M0, x0) and
 * (M1, x2), outputs (hi1^x1^k0, lo1, hi0^x3^k1, lo0); the key is bumped by the
 * Weyl constants between rounds.  A 64-bit-word instance of the same round
 * structure is provided for checking against an independent library.        */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B9u; k1 += 0xBB67AE85u; }
        uint64_t p0 = (uint64_t)0xD2511F53u * x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4])
{
    uint64_t x0 = ctr_in[0], x1 = ctr_in[1], x2 = ctr_in[2], x3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; r++) {
        if (r > 0) { k0 += 0x9E3779B97F4A7C15ull; k1 += 0xBB67AE8584CAA73Bull; }
        unsigned __int128 p0 = (unsigned __int128)0xD2E7470EE14C6C93ull * x0;
        unsigned __int128 p1 = (unsigned __int128)0xCA5A826395121157ull * x2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t y0 = hi1 ^ x1 ^ k0, y1 = lo1, y2 = hi0 ^ x3 ^ k1, y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* 24-bit centred uniform in (0,1): ((r >> 8) + 1/2) 2^-24, exact in binary32. */
double orc_u24(uint32_t r) { return ((double)(r >> 8) + 0.5) * (1.0 / 16777216.0); }

/* Stream layout: key = (seed lo32, seed hi32); counter = (dm index, gas index,
 * step, tag | box << 8).  Tag 0: gas-velocity sample of pair (i,j); tag 1:
 * scattering direction of pair (i,j); tag 2: per-DM decision uniform (gas
 * index 0xFFFFFFFF); tag 5: tilted relative velocity of the chosen pair
 * (Rao-Blackwellised sampling only).                                         */
static void orc_block(uint64_t seed, uint32_t i, uint32_t j, uint32_t step, uint32_t tag, uint32_t box,
                      double u[4])
{
    uint32_t ctr[4] = {i, j, step, tag | (box << 8)};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t r[4];
    orc_philox4x32_10(ctr, key, r);
    for (int k = 0; k < 4; k++) u[k] = orc_u24(r[k]);
}

/* Box-Muller: three standard normals from one block.                        */
void orc_normals3(const double u[4], double z[3])
{
    double r0 = sqrt(-2.0 * log(u[0])), r1 = sqrt(-2.0 * log(u[2]));
    z[0] = r0 * cos(2.0 * ORC_PI * u[1]);
    z[1] = r0 * sin(2.0 * ORC_PI * u[1]);
    z[2] = r1 * cos(2.0 * ORC_PI * u[3]);
}

/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t n;
    const double *pos;        /* [n][3] kpc */
    const double *vel;        /* [n][3] km/s */
    const double *mass;       /* [n] Msun */
    const double *h;          /* [n] kpc (kernel support radius) */
    const double *u;          /* gas: [n] (km/s)^2; ignored for DM */
    const double *mu;         /* gas: [n] g, NULL => proton mass */
    const uint8_t *active;    /* NULL => all active */
    const double *dt;         /* NULL => params dt */
} orc_particles;

typedef struct {
    double sigma0_cm2;
    int n_pow;
    double m_chi_g;
    double dt;
    uint64_t seed;
    uint32_t step;
    uint32_t box_id;
    double box[3];            /* periodic side lengths; 0 => open */
    double aniso_g;           /* dsigma/dOmega = sigma(v) p(Omega): Henyey-Greenstein p with mean
                                 cos theta = g (0: isotropic); sigma-bar = (1 - g) sigma */
    int gas_closure;          /* 1: each gas takes the per-gas Maxwellian closure of its DM neighbours */
    int dm_rb;                /* 1: Rao-Blackwellised DM sampling (expected P_ij, tilted partner draw) */
} orc_params;

enum { ORC_C_PAIRS_GAS = 0, ORC_C_PAIRS_DM, ORC_C_SCATTERS, ORC_C_NEAR_BOUNDARY, ORC_C_NEAR_DECISION,
       ORC_C_CRIT_VIOL, ORC_C_P_GE_1, ORC_C_NONFINITE, ORC_NCOUNTERS };

typedef struct {
    double *dv_dm;            /* [n_dm][3] km/s */
    double *dp_gas;           /* [n_gas][3] Msun km/s */
    double *de_gas;           /* [n_gas] Msun (km/s)^2, internal energy */
    double *dp_abs;           /* [n_gas][3] sum of |terms| (nullable) */
    double *de_abs;           /* [n_gas] (nullable) */
    double *pk_abs;           /* [n_gas] sum over pairs and components of |term| g(0)/g (nullable) */
    int32_t *partner;         /* [n_dm] gas index or -1 */
    double *p_sum;            /* [n_dm] (nullable) */
    double *p_max;            /* [n_dm] (nullable) */
    uint8_t *flags;           /* [n_dm] bit0 near decision, bit1 near-boundary pair (nullable) */
    uint64_t counters[ORC_NCOUNTERS];
} orc_out;

static void min_image(const orc_params *par, double dx[3])
{
    for (int k = 0; k < 3; k++)
        if (par->box[k] > 0.0) dx[k] -= par->box[k] * nearbyint(dx[k] / par->box[k]);
}

/* Pair membership (Appendix D: overlap vanishes iff d >= h_i + h_j).         */
static int pair_test(const orc_particles *gas, const orc_particles *dm, const orc_params *par, int64_t j,
                     int64_t i, double *d_out, int *near)
{
    double dx[3];
    for (int k = 0; k < 3; k++) dx[k] = dm->pos[3 * i + k] - gas->pos[3 * j + k];
    min_image(par, dx);
    double d2 = dx[0] * dx[0] + dx[1] * dx[1] + dx[2] * dx[2];
    double hs = dm->h[i] + gas->h[j];
    double r = d2 / (hs * hs);
    if (near) *near = fabs(r - 1.0) <= 1e-6;
    *d_out = sqrt(d2);
    return d2 < hs * hs;
}

static double gas_mu(const orc_particles *gas, int64_t j) { return gas->mu ? gas->mu[j] : ORC_MP_G; }
static double gas_vs(const orc_particles *gas, int64_t j) { return sqrt(2.0 * gas->u[j] / 3.0); }
static double p_dt(const orc_particles *p, const orc_params *par, int64_t k) { return p->dt ? p->dt[k] : par->dt; }

/* Neumaier-compensated accumulator. */
typedef struct { double s, c; } orc_sum;
static void nsum_add(orc_sum *a, double x)
{
    double t = a->s + x;
    if (fabs(a->s) >= fabs(x)) a->c += (a->s - t) + x; else a->c += (x - t) + a->s;
    a->s = t;
}
static double nsum_get(const orc_sum *a) { return a->s + a->c; }

/* Gas mean field for gas j (eq. gas-dVdt and gas-dTdt):
 *   dV_j/dt = sum_i M_i/(m_chi+mu_j) g_ij A(w) w,
 *   (3/(2 mu_j)) dT_j/dt = sum_i M_i/(m_chi+mu_j) g_ij [w^2 A - mu_j/(m_chi+mu_j) B],
 * w = v_i - V_j.  Output dp = M_j dt_j dV/dt and dE = M_j dt_j (3/(2mu)) dT/dt
 * (the internal-energy change; the bulk-kinetic part is V_j . dp).  Sums run
 * over DM in index order, compensated.  cand: ascending DM candidates (NULL:
 * every DM particle).                                                       */
static uint64_t gas_closure_one(const orc_particles *gas, const orc_particles *dm, const orc_params *par,
                                int64_t j, const int64_t *cand, int64_t ncand, orc_out *out);

static void gas_one(const orc_particles *gas, const orc_particles *dm, const orc_params *par, int64_t j,
                    const int64_t *cand, int64_t ncand, orc_out *out, uint64_t *npairs)
{
    if (par->gas_closure) {
        *npairs += gas_closure_one(gas, dm, par, j, cand, ncand, out);
        return;
    }
    orc_sum sp[3] = {{0, 0}, {0, 0}, {0, 0}}, se = {0, 0};
    double ap[3] = {0, 0, 0}, ae = 0, apk = 0;
    uint64_t np = 0;
    int gas_act = gas->active ? gas->active[j] : 1;
    if (gas_act) {
        double mu = gas_mu(gas, j), vs = gas_vs(gas, j);
        /* the mean field takes the momentum-transfer cross section (eq. scrA, scrB):
         * sigma-bar = int dOmega dsigma/dOmega (1 - cos theta) = (1 - g) sigma */
        double sig_kpc2 = par->sigma0_cm2 / (ORC_KPC_CM * ORC_KPC_CM) * (1.0 - par->aniso_g);
        double cfac = sig_kpc2 * pow(ORC_C_KMS, -par->n_pow);
        double redm = mu / (par->m_chi_g + mu);
        int64_t nc = cand ? ncand : dm->n;
        for (int64_t c = 0; c < nc; c++) {
            int64_t i = cand ? cand[c] : c;
            double d;
            if (!pair_test(gas, dm, par, j, i, &d, NULL)) continue;
            np++;
            double g = orc_overlap(d, dm->h[i], gas->h[j]);
            double w[3], w2 = 0;
            for (int k = 0; k < 3; k++) { w[k] = dm->vel[3 * i + k] - gas->vel[3 * j + k]; w2 += w[k] * w[k]; }
            double A, B;
            orc_rates(par->n_pow, sqrt(w2), vs, &A, &B);
            double num = dm->mass[i] * ORC_MSUN_G / (par->m_chi_g + mu);
            double fac = num * g * cfac;
            for (int k = 0; k < 3; k++) { double t = fac * A * w[k]; nsum_add(&sp[k], t); ap[k] += fabs(t); }
            double tE1 = fac * w2 * A, tE2 = -fac * redm * B;
            nsum_add(&se, tE1);
            nsum_add(&se, tE2);
            ae += fabs(tE1) + fabs(tE2);
            if (out->pk_abs && g > 0.0) {
                double gpk = orc_overlap(0.0, dm->h[i], gas->h[j]);
                apk += (fabs(fac * A) * (fabs(w[0]) + fabs(w[1]) + fabs(w[2])) + fabs(tE1) + fabs(tE2)) * gpk / g;
            }
        }
    }
    double sc = gas_act ? gas->mass[j] * p_dt(gas, par, j) : 0.0;
    for (int k = 0; k < 3; k++) {
        out->dp_gas[3 * j + k] = sc * nsum_get(&sp[k]);
        if (out->dp_abs) out->dp_abs[3 * j + k] = sc * ap[k];
    }
    out->de_gas[j] = sc * nsum_get(&se);
    if (out->de_abs) out->de_abs[j] = sc * ae;
    if (out->pk_abs) out->pk_abs[j] = sc * apk;
    *npairs += np;
}

/* Per-gas Maxwellian closure (Appendix F applied per gas particle): the DM
 * around gas j are taken as one Maxwellian population with the kernel-weighted
 * density rho_j = sum_i M_i g_ij, drift W_j = sum_i M_i g_ij w_ij / rho_j and
 * 1-D dispersion s_X^2 = (sum_i M_i g_ij |w_ij|^2 / rho_j - |W_j|^2) / 3, with
 * w_ij = v_i - V_j over the pairs d_ij < h_i + h_j.  The two-population rates
 * at the combined dispersion vth^2 = varsigma_j^2 + s_X^2 then give
 *   dp_j = M_j dt S_j rho_j A(W_j; vth) W_j,
 *   dE_j = M_j dt S_j rho_j [B (m_X s_X^2 - mu varsigma_j^2)/(m_X + mu)
 *                            + A varsigma_j^2 |W_j|^2] / vth^2,
 * S_j = sigma-bar_0 c^-n / (m_X + mu), the Maxwellian average of the per-pair
 * terms of eq. gas-dVdt / gas-dTdt.  Sums are compensated, in DM-index order.
 * dp_abs / de_abs are condition scales: for dp, f A sum_i M_i g_ij |w_ij,k| /
 * rho (the magnitudes of the summed momentum terms, as for the per-pair mean
 * field); for dE, the magnitudes of its three terms times max(1, <|w|^2> /
 * vth^2), the factor by which the cancellation in s_X^2 = (<|w|^2> - |W|^2)/3
 * magnifies a relative change of the moments (<.> the kernel-weighted mean). */
static uint64_t gas_closure_one(const orc_particles *gas, const orc_particles *dm, const orc_params *par,
                                int64_t j, const int64_t *cand, int64_t ncand, orc_out *out)
{
    orc_sum sr = {0, 0}, sw[3] = {{0, 0}, {0, 0}, {0, 0}}, s2 = {0, 0};
    double swa[3] = {0, 0, 0};
    int gas_act = gas->active ? gas->active[j] : 1;
    uint64_t np = 0;
    for (int k = 0; k < 3; k++) { out->dp_gas[3 * j + k] = 0.0; if (out->dp_abs) out->dp_abs[3 * j + k] = 0.0; }
    out->de_gas[j] = 0.0;
    if (out->de_abs) out->de_abs[j] = 0.0;
    if (out->pk_abs) out->pk_abs[j] = 0.0;
    if (!gas_act) return 0;
    double sc = gas->mass[j] * p_dt(gas, par, j);
    int64_t nc = cand ? ncand : dm->n;
    for (int64_t c = 0; c < nc; c++) {
        int64_t i = cand ? cand[c] : c;
        double d;
        if (!pair_test(gas, dm, par, j, i, &d, NULL)) continue;
        np++;
        double mg = dm->mass[i] * orc_overlap(d, dm->h[i], gas->h[j]), w2 = 0.0;
        for (int k = 0; k < 3; k++) {
            double w = dm->vel[3 * i + k] - gas->vel[3 * j + k];
            nsum_add(&sw[k], mg * w);
            swa[k] += fabs(mg * w);
            w2 += w * w;
        }
        nsum_add(&sr, mg);
        nsum_add(&s2, mg * w2);
    }
    double rho = nsum_get(&sr);
    if (!(rho > 0.0)) return np;
    double W[3], W2 = 0.0;
    for (int k = 0; k < 3; k++) { W[k] = nsum_get(&sw[k]) / rho; W2 += W[k] * W[k]; }
    double mw2 = nsum_get(&s2) / rho, sx2 = fmax(0.0, (mw2 - W2) / 3.0);
    double mu = gas_mu(gas, j), vs = gas_vs(gas, j), vth2 = vs * vs + sx2;
    if (!(vth2 > 0.0) && !(W2 > 0.0)) return np;
    double A, B;
    orc_rates(par->n_pow, sqrt(W2), sqrt(vth2), &A, &B);
    double cfac = par->sigma0_cm2 / (ORC_KPC_CM * ORC_KPC_CM) * (1.0 - par->aniso_g) * pow(ORC_C_KMS, -par->n_pow);
    double f = sc * rho * ORC_MSUN_G / (par->m_chi_g + mu) * cfac;
    for (int k = 0; k < 3; k++) {
        out->dp_gas[3 * j + k] = f * A * W[k];
        if (out->dp_abs) out->dp_abs[3 * j + k] = fabs(f * A) * swa[k] / rho;
    }
    if (!(vth2 > 0.0)) {
        /* both populations cold: the limit of either order is the per-pair form
         * W^2 A - mu/(m_X + mu) B at A = |W|^{n+1}, B = |W|^{n+3}            */
        double e1 = A * W2, e2 = B * mu / (par->m_chi_g + mu);
        out->de_gas[j] = f * (e1 - e2);
        if (out->de_abs) out->de_abs[j] = fabs(f) * (fabs(e1) + fabs(e2));
        return np;
    }
    double e1 = B * par->m_chi_g * sx2 / (par->m_chi_g + mu), e2 = B * mu * vs * vs / (par->m_chi_g + mu);
    double e3 = A * vs * vs * W2;
    out->de_gas[j] = f * (e1 - e2 + e3) / vth2;
    if (out->de_abs) out->de_abs[j] = fabs(f) * (fabs(e1) + fabs(e2) + fabs(e3)) / vth2 * fmax(1.0, mw2 / vth2);
    return np;
}

/* Relative velocity v_i - v^B_ij with v^B_ij = V_j + varsigma_j z, z from the
 * tag-0 block of pair (i,j) (one Maxwellian sample per pair, Sec. 2.2).      */
static void pair_urel(const orc_particles *gas, const orc_particles *dm, const orc_params *par, int64_t j,
                      int64_t i, double urel[3])
{
    double u[4], z[3];
    orc_block(par->seed, (uint32_t)i, (uint32_t)j, par->step, 0u, par->box_id, u);
    orc_normals3(u, z);
    double vs = gas_vs(gas, j);
    for (int k = 0; k < 3; k++) urel[k] = dm->vel[3 * i + k] - (gas->vel[3 * j + k] + vs * z[k]);
}

/* ------------------------------------------------------------------------- */
/* Rao-Blackwellised DM sampling (a variant of Sec. 2.2 that is exact in law;
 * not the paper's scheme).  Pair (i,j) takes the expectation of its
 * scattering probability over the Maxwellian gas-velocity sample,
 *   Pbar_ij = (M_j/mu_j) g_ij sigma0 c^-n dt_i E|w - varsigma_j z|^{n+1},
 * w = v_i - V_j, z ~ N(0, I).  For u ~ N(w, varsigma^2 I), E|u|^{n+3} is the
 * Bhat integral of power n (eq. scrB without sigma0 c^-n), so E|u|^{n+1} is
 * Bhat of power n - 2 (finite for n > -4).  A DM that scatters with partner
 * j draws its relative velocity from the tilted law
 *   p(u) ~ |u|^{n+1} N(u; w, varsigma^2 I),
 * the law of u given a scatter with j in the per-pair scheme; so partner and
 * u have the per-pair scheme's joint distribution whenever P_i <= 1.  The
 * draw is by inversion from the tag-5 block (u0, u1, u2) of the pair: in
 * units of varsigma, r = |u| has density proportional to
 *   r^{n+2} e^{-(r-a)^2/2} (1 - e^{-2 r a}) / (2a),  a = |w|/varsigma
 * (r^{n+3} e^{-r^2/2} at a = 0), inverted at u0 (lower CDF for u0 <= 1/2,
 * upper tail otherwise); given r, c = cos(u, w) has density ~ e^{r a c} on
 * [-1, 1], inverted at u1 (1 - c = -ln(1 - u1 (1 - e^{-2ra})) / (ra)); the
 * azimuth is 2 pi u2 in the frame basis_around(w/|w|) (the z axis if w = 0).
 * Cold gas (varsigma = 0) gives u = w.  The radial CDF is integrated here by
 * adaptive 20-point Gauss-Legendre (nodes from Newton on P_20; halves
 * until two levels agree to 4e-15, at most 8 levels deep) and inverted by
 * bisection to the last bit.                                           */
static void basis_around(const double n[3], double e1[3], double e2[3]);
static double rb_gl_x[20], rb_gl_w[20];
static int rb_gl_ready = 0;

static void rb_gl_init(void)
{
    if (__atomic_load_n(&rb_gl_ready, __ATOMIC_ACQUIRE)) return;
#pragma omp critical(orc_rb_gl)
    {
    if (!rb_gl_ready) {
    const int K = 20;
    for (int i = 0; i < K; i++) {
        double x = cos(ORC_PI * (i + 0.75) / (K + 0.5)), dp = 1.0;
        for (int it = 0; it < 200; it++) {
            double pm = 1.0, pk = x;
            for (int k = 2; k <= K; k++) { double pn = ((2 * k - 1) * x * pk - (k - 1) * pm) / k; pm = pk; pk = pn; }
            dp = K * (pm - x * pk) / (1.0 - x * x);
            double dx = pk / dp;
            x -= dx;
            if (fabs(dx) <= 1e-17) break;
        }
        double pm = 1.0, pk = x;
        for (int k = 2; k <= K; k++) { double pn = ((2 * k - 1) * x * pk - (k - 1) * pm) / k; pm = pk; pk = pn; }
        dp = K * (pm - x * pk) / (1.0 - x * x);
        rb_gl_x[i] = x;
        rb_gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    __atomic_store_n(&rb_gl_ready, 1, __ATOMIC_RELEASE);
    }
    }
}

/* radial density of the tilted law (unnormalised), m = n + 1 */
static double rb_radial(int m, double a, double r)
{
    if (!(r > 0.0)) return 0.0;
    double sh = a > 0.0 ? -expm1(-2.0 * r * a) / (2.0 * a) : r;
    return pow(r, m + 1) * exp(-0.5 * (r - a) * (r - a)) * sh;
}

static double rb_gl(int m, double a, double lo, double hi)
{
    double c = 0.5 * (lo + hi), h = 0.5 * (hi - lo), s = 0.0;
    for (int k = 0; k < 20; k++) s += rb_gl_w[k] * rb_radial(m, a, c + h * rb_gl_x[k]);
    return s * h;
}

static double rb_adapt(int m, double a, double lo, double hi, double whole, int depth)
{
    double mid = 0.5 * (lo + hi);
    double l = rb_gl(m, a, lo, mid), r = rb_gl(m, a, mid, hi);
    /* below width 24/2^8 the 20-point rule is exact to rounding for this integrand (unit scale) */
    if (depth >= 8 || fabs(l + r - whole) <= 4e-15 * fabs(l + r)) return l + r;
    return rb_adapt(m, a, lo, mid, l, depth + 1) + rb_adapt(m, a, mid, hi, r, depth + 1);
}

static double rb_int(int m, double a, double lo, double hi)
{
    if (!(hi > lo)) return 0.0;
    return rb_adapt(m, a, lo, hi, rb_gl(m, a, lo, hi), 0);
}

/* r = |u| / varsigma of the tilted law at uniform u0; support [max(0, a - 12), a + 12] */
double orc_rb_radius(int m, double a, double u0)
{
    rb_gl_init();
    double lo = fmax(0.0, a - 12.0), hi = a + 12.0;
    double Z = rb_int(m, a, lo, hi);
    double bl = lo, bh = hi;
    if (u0 <= 0.5) {
        double T = u0 * Z;
        for (int it = 0; it < 200; it++) {
            double mid = 0.5 * (bl + bh);
            if (!(mid > bl && mid < bh)) break;
            if (rb_int(m, a, lo, mid) < T) bl = mid; else bh = mid;
        }
    } else {
        double T = (1.0 - u0) * Z;
        for (int it = 0; it < 200; it++) {
            double mid = 0.5 * (bl + bh);
            if (!(mid > bl && mid < bh)) break;
            if (rb_int(m, a, mid, hi) > T) bl = mid; else bh = mid;
        }
    }
    return 0.5 * (bl + bh);
}

/* the tilted relative velocity for w (km/s), varsigma vs, power n, uniforms u[0..2] */
void orc_rb_urel(int n, const double w[3], double vs, const double u[3], double urel[3])
{
    double wn = sqrt(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
    if (!(vs > 0.0)) { for (int k = 0; k < 3; k++) urel[k] = w[k]; return; }
    double a = wn / vs;
    double r = orc_rb_radius(n + 1, a, u[0]);
    double kap = r * a;
    double omc = kap > 0.0 ? -log1p(u[1] * expm1(-2.0 * kap)) / kap : 2.0 * u[1];  /* 1 - cos */
    double c = 1.0 - omc, s = sqrt(fmax(0.0, omc * (2.0 - omc)));
    double e[3] = {0.0, 0.0, 1.0}, e1[3], e2[3];
    if (wn > 0.0) for (int k = 0; k < 3; k++) e[k] = w[k] / wn;
    basis_around(e, e1, e2);
    double ph = 2.0 * ORC_PI * u[2];
    for (int k = 0; k < 3; k++) urel[k] = vs * r * (c * e[k] + s * (cos(ph) * e1[k] + sin(ph) * e2[k]));
}

/* Scattering probability P_ij = (M_j/mu_j) g_ij sigma(v_rel) v_rel dt_i
 * (eq. dm-update-prob), sigma = sigma0 (v/c)^n.  Rao-Blackwellised: the
 * expectation over the gas-velocity sample (urel is then set by dm_one).    */
static double pair_P(const orc_particles *gas, const orc_particles *dm, const orc_params *par, int64_t j,
                     int64_t i, double d, double urel[3])
{
    if (par->dm_rb) {
        double w2 = 0.0, A, Bm;
        for (int k = 0; k < 3; k++) {
            double w = dm->vel[3 * i + k] - gas->vel[3 * j + k];
            w2 += w * w;
            urel[k] = 0.0;
        }
        orc_rates(par->n_pow - 2, sqrt(w2), gas_vs(gas, j), &A, &Bm);
        double g = orc_overlap(d, dm->h[i], gas->h[j]);
        double ncount = gas->mass[j] * ORC_MSUN_G / gas_mu(gas, j);
        double sig = par->sigma0_cm2 / (ORC_KPC_CM * ORC_KPC_CM) * pow(ORC_C_KMS, -par->n_pow);
        return ncount * g * sig * Bm * p_dt(dm, par, i);
    }
    pair_urel(gas, dm, par, j, i, urel);
    double vrel = sqrt(urel[0] * urel[0] + urel[1] * urel[1] + urel[2] * urel[2]);
    double g = orc_overlap(d, dm->h[i], gas->h[j]);
    double ncount = gas->mass[j] * ORC_MSUN_G / gas_mu(gas, j);
    double sig = par->sigma0_cm2 / (ORC_KPC_CM * ORC_KPC_CM) * pow(vrel / ORC_C_KMS, par->n_pow);
    return ncount * g * sig * vrel * p_dt(dm, par, i);
}

typedef struct { int64_t j; double P; double urel[3]; } orc_pair;

/* Henyey-Greenstein scattering angle (Sec. 2.2-2.3 with p(Omega) of mean
 * cos theta = g): the density of c = cos theta is (1 - g^2) / (2 (1 + g^2 -
 * 2 g c)^{3/2}) on [-1, 1]; its CDF F(c) = (1 - g^2) / (2g) [(1 + g^2 -
 * 2 g c)^{-1/2} - 1/(1 + g)] set equal to u and solved for c.  Written as a
 * ratio of polynomials in t = 2u - 1 (no division by g), so g -> 0 gives t.
 * sin theta from 1 - c^2 in factored form, 4 (1 - g^2)^2 u (1 - u)
 * (1 - g + g u) (1 + g u) / (1 + g t)^4, accurate where c is near +-1.     */
static void hg_inverse_cdf(double g, double u, double *ct, double *st)
{
    double t = 2.0 * u - 1.0, den = 1.0 + g * t;
    double c = (2.0 * t + g * (t * t + 3.0) + 2.0 * g * g * t + g * g * g * (t * t - 1.0)) / (2.0 * den * den);
    *ct = fmax(-1.0, fmin(1.0, c));
    double p = u * (1.0 - u) * (1.0 - g + g * u) * (1.0 + g * u);
    *st = 2.0 * (1.0 - g * g) * sqrt(fmax(0.0, p)) / (den * den);
}

/* Unit vectors e1, e2 perpendicular to the unit vector n and to each other
 * (Duff et al., Building an orthonormal basis, revisited, JCGT 2017). */
static void basis_around(const double n[3], double e1[3], double e2[3])
{
    double sg = n[2] >= 0.0 ? 1.0 : -1.0;
    double a = -1.0 / (sg + n[2]), b = n[0] * n[1] * a;
    e1[0] = 1.0 + sg * n[0] * n[0] * a; e1[1] = sg * b; e1[2] = -sg * n[0];
    e2[0] = b; e2[1] = sg + n[1] * n[1] * a; e2[2] = -n[1];
}

static int cmp_pair(const void *x, const void *y)
{
    int64_t a = ((const orc_pair *)x)->j, b = ((const orc_pair *)y)->j;
    return (a > b) - (a < b);
}

/* DM Monte Carlo for DM i (eq. dm-update-vels, dm-update-prob; Sec. 2.4):
 * one categorical draw from nu'_i: U_i from the tag-2 block; if U_i < P_i =
 * sum_j P_ij the partner is the first gas index (ascending) whose running sum
 * exceeds U_i; the new direction is isotropic (tag-1 block of the chosen
 * pair, cos theta = 2u0-1, phi = 2 pi u1) and the kick follows eq. scatter_chi
 * with the same gas-velocity sample that set P_ij.  Criterion of eq.
 * prob_criterion is counted, not enforced.  cand: ascending gas candidates
 * (NULL: every gas particle); a near-boundary pair must be among them.      */
static void dm_one(const orc_particles *gas, const orc_particles *dm, const orc_params *par, int64_t i,
                   const int64_t *cand, int64_t ncand, orc_out *out, uint64_t cnt[ORC_NCOUNTERS])
{
    for (int k = 0; k < 3; k++) out->dv_dm[3 * i + k] = 0.0;
    out->partner[i] = -1;
    if (out->p_sum) out->p_sum[i] = 0.0;
    if (out->p_max) out->p_max[i] = 0.0;
    if (out->flags) out->flags[i] = 0;
    if (dm->active && !dm->active[i]) return;

    size_t cap = 64, np = 0;
    orc_pair *pairs = (orc_pair *)malloc(cap * sizeof(orc_pair));
    int near_b = 0;
    int64_t nc = cand ? ncand : gas->n;
    for (int64_t c = 0; c < nc; c++) {
        int64_t j = cand ? cand[c] : c;
        double d;
        int near;
        int in = pair_test(gas, dm, par, j, i, &d, &near);
        if (near) near_b = 1;
        if (!in) continue;
        if (np == cap) { cap *= 2; pairs = (orc_pair *)realloc(pairs, cap * sizeof(orc_pair)); }
        pairs[np].j = j;
        pairs[np].P = pair_P(gas, dm, par, j, i, d, pairs[np].urel);
        np++;
    }
    qsort(pairs, np, sizeof(orc_pair), cmp_pair); /* already ascending; kept explicit */
    double S = 0.0, pmax = 0.0;
    int nonfinite = 0;
    for (size_t k = 0; k < np; k++) {
        double P = pairs[k].P;
        if (!isfinite(P)) nonfinite = 1;
        S += P;
        if (P > pmax) pmax = P;
        double mu = gas_mu(gas, pairs[k].j);
        double q = (par->m_chi_g + mu) / mu;
        double crit = fmin(0.1, 1e-4 * q * q);
        if (P >= crit) cnt[ORC_C_CRIT_VIOL]++;
    }
    cnt[ORC_C_PAIRS_DM] += np;
    if (nonfinite) cnt[ORC_C_NONFINITE]++;
    if (S >= 1.0) cnt[ORC_C_P_GE_1]++;
    if (near_b) cnt[ORC_C_NEAR_BOUNDARY]++;
    if (out->p_sum) out->p_sum[i] = S;
    if (out->p_max) out->p_max[i] = pmax;

    double ud[4];
    orc_block(par->seed, (uint32_t)i, 0xFFFFFFFFu, par->step, 2u, par->box_id, ud);
    double U = ud[0];
    int near_d = fabs(S - U) <= 1e-6 * U;
    int64_t jstar = -1;
    size_t kstar = 0;
    if (U < S) {
        double run = 0.0;
        for (size_t k = 0; k < np; k++) {
            run += pairs[k].P;
            if (fabs(run - U) <= 1e-6 * U) near_d = 1;
            if (jstar < 0 && run > U) { jstar = pairs[k].j; kstar = k; }
        }
        if (jstar < 0 && np > 0) { jstar = pairs[np - 1].j; kstar = np - 1; }
    }
    if (near_d) cnt[ORC_C_NEAR_DECISION]++;
    if (out->flags) out->flags[i] = (uint8_t)((near_d ? 1 : 0) | (near_b ? 2 : 0));
    if (jstar >= 0) {
        cnt[ORC_C_SCATTERS]++;
        out->partner[i] = (int32_t)jstar;
        double *ur = pairs[kstar].urel;
        if (par->dm_rb) {
            double ut[4], w[3];
            orc_block(par->seed, (uint32_t)i, (uint32_t)jstar, par->step, 5u, par->box_id, ut);
            for (int k = 0; k < 3; k++) w[k] = dm->vel[3 * i + k] - gas->vel[3 * jstar + k];
            orc_rb_urel(par->n_pow, w, gas_vs(gas, jstar), ut, ur);
        }
        double vrel = sqrt(ur[0] * ur[0] + ur[1] * ur[1] + ur[2] * ur[2]);
        if (vrel > 0.0) {
            double ua[4];
            orc_block(par->seed, (uint32_t)i, (uint32_t)jstar, par->step, 1u, par->box_id, ua);
            double ph = 2.0 * ORC_PI * ua[1];
            double nn[3];
            if (par->aniso_g == 0.0) {
                /* isotropic: the new direction itself, cos theta about the z axis */
                double ct = 2.0 * ua[0] - 1.0, st = sqrt(fmax(0.0, 1.0 - ct * ct));
                nn[0] = st * cos(ph); nn[1] = st * sin(ph); nn[2] = ct;
            } else {
                /* scattering angle theta about the incoming relative velocity, from p(Omega) */
                double uh[3] = {ur[0] / vrel, ur[1] / vrel, ur[2] / vrel}, e1[3], e2[3];
                double ct, st;
                hg_inverse_cdf(par->aniso_g, ua[0], &ct, &st);
                basis_around(uh, e1, e2);
                for (int k = 0; k < 3; k++) nn[k] = ct * uh[k] + st * (cos(ph) * e1[k] + sin(ph) * e2[k]);
            }
            double mu = gas_mu(gas, jstar);
            double fr = mu / (par->m_chi_g + mu);
            for (int k = 0; k < 3; k++) out->dv_dm[3 * i + k] = fr * vrel * (nn[k] - ur[k] / vrel);
        }
    }
    free(pairs);
}

/* ------------------------------------------------------------------------- */
/* Candidate search on uniform grids (a filter only: the pair set is defined by
 * pair_test).  The particles of one species are split into levels by kernel
 * radius, level l holding h in [2^l h_min, 2^(l+1) h_min); each level is
 * bucketed on a uniform grid whose cell side c_l >= 2^(l+1) h_min, as cell
 * keys sorted with their particle indices.  A query point x with radius h_x
 * receives every particle of every level whose cell lies within
 * (h_x + c_l)(1 + 1e-5) of x per axis (each periodic image once), or the
 * whole level when that box covers more cells than the level has particles.
 * Candidates come back sorted by index.                                    */
#define ORC_GRID_LEVELS 48
typedef struct {
    int64_t n;                /* particles in the level */
    int64_t *idx;             /* particle indices, sorted by cell key */
    uint64_t *key;            /* their cell keys */
    int64_t nc[3];            /* cells per axis */
    double cs[3];             /* cell sides */
    double org[3];            /* grid origin */
    double hmax;              /* largest h in the level */
} orc_level;

typedef struct {
    int nlev;
    orc_level lev[ORC_GRID_LEVELS];
    double box[3];            /* periodic sides; 0 => open */
} orc_grid;

typedef struct { uint64_t k; int64_t i; } orc_kv;
static int cmp_kv(const void *a, const void *b)
{
    uint64_t x = ((const orc_kv *)a)->k, y = ((const orc_kv *)b)->k;
    if (x != y) return (x > y) - (x < y);
    int64_t u = ((const orc_kv *)a)->i, v = ((const orc_kv *)b)->i;
    return (u > v) - (u < v);
}
static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static double wrap(double x, double L) { return L > 0.0 ? x - L * floor(x / L) : x; }

static void grid_build(orc_grid *g, const orc_particles *p, const orc_params *par)
{
    memset(g, 0, sizeof(*g));
    for (int k = 0; k < 3; k++) g->box[k] = par->box[k];
    if (p->n == 0) return;
    double hmin = INFINITY;
    for (int64_t i = 0; i < p->n; i++) if (p->h[i] > 0.0 && p->h[i] < hmin) hmin = p->h[i];
    if (!(hmin < INFINITY)) hmin = 1.0;
    int *lv = (int *)malloc((size_t)p->n * sizeof(int));
    int64_t cnt[ORC_GRID_LEVELS] = {0};
    for (int64_t i = 0; i < p->n; i++) {
        int l = p->h[i] > hmin ? (int)floor(log2(p->h[i] / hmin)) : 0;
        if (l < 0) l = 0;
        if (l >= ORC_GRID_LEVELS) l = ORC_GRID_LEVELS - 1;
        lv[i] = l;
        cnt[l]++;
        if (l + 1 > g->nlev) g->nlev = l + 1;
    }
    for (int l = 0; l < g->nlev; l++) {
        orc_level *L = &g->lev[l];
        L->n = cnt[l];
        if (L->n == 0) continue;
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        L->hmax = 0.0;
        for (int64_t i = 0; i < p->n; i++) {
            if (lv[i] != l) continue;
            if (p->h[i] > L->hmax) L->hmax = p->h[i];
            for (int k = 0; k < 3; k++) {
                double x = wrap(p->pos[3 * i + k], g->box[k]);
                if (x < lo[k]) lo[k] = x;
                if (x > hi[k]) hi[k] = x;
            }
        }
        double c = ldexp(hmin, l + 1);
        if (L->hmax > c) c = L->hmax;
        for (int k = 0; k < 3; k++) {
            if (g->box[k] > 0.0) {
                int64_t n = (int64_t)floor(g->box[k] / c);
                L->nc[k] = n < 1 ? 1 : (n > 2097151 ? 2097151 : n);
                L->cs[k] = g->box[k] / (double)L->nc[k];
                L->org[k] = 0.0;
            } else {
                int64_t n = (int64_t)floor((hi[k] - lo[k]) / c) + 1;
                L->nc[k] = n < 1 ? 1 : (n > 2097151 ? 2097151 : n);
                L->cs[k] = c;
                L->org[k] = lo[k];
            }
        }
        orc_kv *kv = (orc_kv *)malloc((size_t)L->n * sizeof(orc_kv));
        int64_t m = 0;
        for (int64_t i = 0; i < p->n; i++) {
            if (lv[i] != l) continue;
            int64_t ci[3];
            for (int k = 0; k < 3; k++) {
                int64_t t = (int64_t)floor((wrap(p->pos[3 * i + k], g->box[k]) - L->org[k]) / L->cs[k]);
                ci[k] = t < 0 ? 0 : (t >= L->nc[k] ? L->nc[k] - 1 : t);
            }
            kv[m].k = ((uint64_t)ci[0] * (uint64_t)L->nc[1] + (uint64_t)ci[1]) * (uint64_t)L->nc[2] + (uint64_t)ci[2];
            kv[m].i = i;
            m++;
        }
        qsort(kv, (size_t)L->n, sizeof(orc_kv), cmp_kv);
        L->idx = (int64_t *)malloc((size_t)L->n * sizeof(int64_t));
        L->key = (uint64_t *)malloc((size_t)L->n * sizeof(uint64_t));
        for (int64_t t = 0; t < L->n; t++) { L->idx[t] = kv[t].i; L->key[t] = kv[t].k; }
        free(kv);
    }
    free(lv);
}

static void grid_free(orc_grid *g)
{
    for (int l = 0; l < g->nlev; l++) { free(g->lev[l].idx); free(g->lev[l].key); }
}

typedef struct { int64_t *v; int64_t n, cap; } orc_list;
static void list_push(orc_list *a, int64_t x)
{
    if (a->n == a->cap) {
        a->cap = a->cap ? 2 * a->cap : 256;
        a->v = (int64_t *)realloc(a->v, (size_t)a->cap * sizeof(int64_t));
    }
    a->v[a->n++] = x;
}

static int64_t lower_key(const uint64_t *key, int64_t n, uint64_t k)
{
    int64_t lo = 0, hi = n;
    while (lo < hi) { int64_t mid = (lo + hi) / 2; if (key[mid] < k) lo = mid + 1; else hi = mid; }
    return lo;
}

/* Cell range along one axis for [x - R, x + R]: cells lo..hi (hi - lo + 1 <=
 * nc; with wrap, indices are taken modulo nc).                              */
static void axis_range(const orc_level *L, int k, double x, double R, int periodic, int64_t *lo, int64_t *hi)
{
    double a = (x - R - L->org[k]) / L->cs[k], b = (x + R - L->org[k]) / L->cs[k];
    int64_t i0 = (int64_t)floor(a), i1 = (int64_t)floor(b);
    if (periodic) {
        if (i1 - i0 + 1 >= L->nc[k]) { i0 = 0; i1 = L->nc[k] - 1; }
    } else {
        if (i0 < 0) i0 = 0;
        if (i1 > L->nc[k] - 1) i1 = L->nc[k] - 1;
    }
    *lo = i0;
    *hi = i1;
}

static int64_t wrapi(int64_t i, int64_t n) { int64_t r = i % n; return r < 0 ? r + n : r; }

static void grid_query(const orc_grid *g, const double x[3], double hx, orc_list *out)
{
    out->n = 0;
    for (int l = 0; l < g->nlev; l++) {
        const orc_level *L = &g->lev[l];
        if (L->n == 0) continue;
        double R = (hx + L->hmax) * (1.0 + 1e-5) + 1e-12 * (fabs(x[0]) + fabs(x[1]) + fabs(x[2]) + 1.0);
        int64_t lo[3], hi[3];
        double xw[3];
        double ncell = 1.0;
        int empty = 0;
        for (int k = 0; k < 3; k++) {
            int per = g->box[k] > 0.0;
            xw[k] = wrap(x[k], g->box[k]);
            axis_range(L, k, xw[k], R, per, &lo[k], &hi[k]);
            if (hi[k] < lo[k]) empty = 1;
            ncell *= (double)(hi[k] - lo[k] + 1);
        }
        if (empty) continue;
        if (ncell > (double)L->n) {          /* cheaper to take the whole level */
            for (int64_t t = 0; t < L->n; t++) list_push(out, L->idx[t]);
            continue;
        }
        for (int64_t ix = lo[0]; ix <= hi[0]; ix++)
            for (int64_t iy = lo[1]; iy <= hi[1]; iy++) {
                uint64_t base = ((uint64_t)wrapi(ix, L->nc[0]) * (uint64_t)L->nc[1] + (uint64_t)wrapi(iy, L->nc[1])) *
                                (uint64_t)L->nc[2];
                /* z run(s): contiguous keys, split where a periodic range wraps */
                int64_t z0 = lo[2], z1 = hi[2];
                int64_t runs[2][2];
                int nr = 0;
                if (wrapi(z0, L->nc[2]) <= wrapi(z1, L->nc[2]) && z1 - z0 + 1 < L->nc[2] + 1 &&
                    wrapi(z0, L->nc[2]) + (z1 - z0) < L->nc[2]) {
                    runs[0][0] = wrapi(z0, L->nc[2]); runs[0][1] = runs[0][0] + (z1 - z0); nr = 1;
                } else {
                    runs[0][0] = wrapi(z0, L->nc[2]); runs[0][1] = L->nc[2] - 1;
                    runs[1][0] = 0; runs[1][1] = wrapi(z1, L->nc[2]); nr = 2;
                }
                for (int r = 0; r < nr; r++) {
                    int64_t a = lower_key(L->key, L->n, base + (uint64_t)runs[r][0]);
                    int64_t b = lower_key(L->key, L->n, base + (uint64_t)runs[r][1] + 1);
                    for (int64_t t = a; t < b; t++) list_push(out, L->idx[t]);
                }
            }
    }
    qsort(out->v, (size_t)out->n, sizeof(int64_t), cmp_i64);
}

/* Full step for selected owners.  gas_sel/dm_sel list the owner indices to
 * evaluate (NULL => all).  Outputs of unselected owners are left untouched. */
static int step_impl(const orc_particles *gas, const orc_particles *dm, const orc_params *par, orc_out *out,
                     const int64_t *gas_sel, int64_t n_gas_sel, const int64_t *dm_sel, int64_t n_dm_sel, int use_grid)
{
    if (!gas || !dm || !par || !out) return -1;
    memset(out->counters, 0, sizeof(out->counters));
    int64_t ng = gas_sel ? n_gas_sel : gas->n;
    int64_t nd = dm_sel ? n_dm_sel : dm->n;
    orc_grid *gg = NULL, *gd = NULL;   /* grids over gas and over DM */
    if (use_grid) {
        gg = (orc_grid *)malloc(sizeof(orc_grid));
        gd = (orc_grid *)malloc(sizeof(orc_grid));
        grid_build(gg, gas, par);
        grid_build(gd, dm, par);
    }
    uint64_t pg = 0;
#pragma omp parallel reduction(+ : pg)
    {
        orc_list cl = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < ng; t++) {
            int64_t j = gas_sel ? gas_sel[t] : t;
            if (gd) grid_query(gd, gas->pos + 3 * j, gas->h[j], &cl);
            gas_one(gas, dm, par, j, gd ? cl.v : NULL, cl.n, out, &pg);
        }
        free(cl.v);
    }
    out->counters[ORC_C_PAIRS_GAS] = pg;
    uint64_t c[ORC_NCOUNTERS];
    memset(c, 0, sizeof(c));
    uint64_t c1 = 0, c2 = 0, c3 = 0, c4 = 0, c5 = 0, c6 = 0, c7 = 0;
#pragma omp parallel reduction(+ : c1, c2, c3, c4, c5, c6, c7)
    {
        orc_list ca = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 16)
        for (int64_t t = 0; t < nd; t++) {
            int64_t i = dm_sel ? dm_sel[t] : t;
            uint64_t cl[ORC_NCOUNTERS];
            memset(cl, 0, sizeof(cl));
            if (gg) grid_query(gg, dm->pos + 3 * i, dm->h[i], &ca);
            dm_one(gas, dm, par, i, gg ? ca.v : NULL, ca.n, out, cl);
            c1 += cl[ORC_C_PAIRS_DM]; c2 += cl[ORC_C_SCATTERS]; c3 += cl[ORC_C_NEAR_BOUNDARY];
            c4 += cl[ORC_C_NEAR_DECISION]; c5 += cl[ORC_C_CRIT_VIOL]; c6 += cl[ORC_C_P_GE_1];
            c7 += cl[ORC_C_NONFINITE];
        }
        free(ca.v);
    }
    if (use_grid) { grid_free(gg); grid_free(gd); free(gg); free(gd); }
    out->counters[ORC_C_PAIRS_DM] = c1; out->counters[ORC_C_SCATTERS] = c2;
    out->counters[ORC_C_NEAR_BOUNDARY] = c3; out->counters[ORC_C_NEAR_DECISION] = c4;
    out->counters[ORC_C_CRIT_VIOL] = c5; out->counters[ORC_C_P_GE_1] = c6; out->counters[ORC_C_NONFINITE] = c7;
    (void)c;
    return 0;
}

int orc_step_sel(const orc_particles *gas, const orc_particles *dm, const orc_params *par, orc_out *out,
                 const int64_t *gas_sel, int64_t n_gas_sel, const int64_t *dm_sel, int64_t n_dm_sel)
{
    return step_impl(gas, dm, par, out, gas_sel, n_gas_sel, dm_sel, n_dm_sel, 0);
}

/* The same step with candidates from the uniform grids (identical results). */
int orc_step_sel_grid(const orc_particles *gas, const orc_particles *dm, const orc_params *par, orc_out *out,
                      const int64_t *gas_sel, int64_t n_gas_sel, const int64_t *dm_sel, int64_t n_dm_sel)
{
    return step_impl(gas, dm, par, out, gas_sel, n_gas_sel, dm_sel, n_dm_sel, 1);
}

int orc_step(const orc_particles *gas, const orc_particles *dm, const orc_params *par, orc_out *out)
{
    return orc_step_sel(gas, dm, par, out, NULL, 0, NULL, 0);
}

/* Brute-force pair set (Appendix D support; each unordered pair once):
 * writes up to cap (dm index, gas index) pairs in (dm, gas) order and
 * returns the total count.                                                   */
int64_t orc_pairs(const orc_particles *gas, const orc_particles *dm, const orc_params *par, int64_t *out_i,
                  int64_t *out_j, int64_t cap)
{
    int64_t cnt = 0;
    for (int64_t i = 0; i < dm->n; i++)
        for (int64_t j = 0; j < gas->n; j++) {
            double d;
            if (pair_test(gas, dm, par, j, i, &d, NULL)) {
                if (cnt < cap) { out_i[cnt] = i; out_j[cnt] = j; }
                cnt++;
            }
        }
    return cnt;
}

/* Active sets of one step of a hierarchical-timestep run (reading of the
 * Milky-Way-scale setup: an independent fraction of each species active per
 * step): particle i of species s (0 gas, 1 DM) is active iff the first
 * uniform of the block (i, s, step, tag 3) lies below frac.               */
void orc_active_flags(int64_t n, uint32_t species, uint32_t step, uint64_t seed, uint32_t box, double frac,
                      uint8_t *out)
{
    for (int64_t i = 0; i < n; i++) {
        double u[4];
        orc_block(seed, (uint32_t)i, species, step, 3u, box, u);
        out[i] = u[0] < frac ? 1 : 0;
    }
}

/* Per-owner pair statistics for selected owners (the same pair set as
 * orc_pairs, brute force over the other species): for owner sel[t] (a gas
 * index when owner_is_dm == 0, else a DM index) the number of partners, the
 * sum of their indices and the sum of their squared indices; use_grid takes
 * the candidates from the uniform grids (same sets).                        */
void orc_pair_stats(const orc_particles *gas, const orc_particles *dm, const orc_params *par, const int64_t *sel,
                    int64_t nsel, int owner_is_dm, int use_grid, int64_t *cnt, uint64_t *sum1, uint64_t *sum2)
{
    orc_grid *g = NULL;
    if (use_grid) {
        g = (orc_grid *)malloc(sizeof(orc_grid));
        grid_build(g, owner_is_dm ? gas : dm, par);
    }
#pragma omp parallel
    {
    orc_list cl = {NULL, 0, 0};
#pragma omp for schedule(dynamic, 4)
    for (int64_t t = 0; t < nsel; t++) {
        int64_t o = sel[t], n = 0;
        uint64_t s1 = 0, s2 = 0;
        const orc_particles *own = owner_is_dm ? dm : gas;
        if (g) grid_query(g, own->pos + 3 * o, own->h[o], &cl);
        int64_t nother = g ? cl.n : (owner_is_dm ? gas->n : dm->n);
        for (int64_t c = 0; c < nother; c++) {
            int64_t k = g ? cl.v[c] : c;
            double d;
            int in = owner_is_dm ? pair_test(gas, dm, par, k, o, &d, NULL) : pair_test(gas, dm, par, o, k, &d, NULL);
            if (!in) continue;
            n++;
            s1 += (uint64_t)k;
            s2 += (uint64_t)k * (uint64_t)k;
        }
        cnt[t] = n;
        sum1[t] = s1;
        sum2[t] = s2;
    }
    free(cl.v);
    }
    if (g) { grid_free(g); free(g); }
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
