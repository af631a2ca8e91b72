// dmb_device.h -- device-side math of the DM-gas pair step for gfx950.
//
// Paper: Hainje & Farrar, arXiv 2603.24688.  Each function names the passage
// it implements.  Templates over float/double are one code path: the pair
// math runs in `Real`, positions and sums in double.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace dmb {

constexpr double kPi = 3.14159265358979323846;
constexpr double kSqrtPi = 1.7724538509055160273;

// ---------------------------------------------------------------------------
// Cubic-spline kernel (Sec. 2.4): w(q) = 8/pi {1-6q^2+6q^3; 2(1-q)^3; 0}.
template <typename T>
__device__ __forceinline__ T kernel_w(T q)
{
    const T c = T(8.0 / kPi);
    if (q <= T(0.5)) return c * (T(1) + q * q * (T(6) * q - T(6)));
    if (q < T(1)) { T p = T(1) - q; return c * T(2) * p * p * p; }
    return T(0);
}

// psi(Q) = int_0^Q q w(q) dq differences on one polynomial branch, factored so
// that a small b - a keeps relative accuracy (Appendix D inner integral).
__device__ __forceinline__ double psi_piece(int br, double a, double b, double bma)
{
    const double c = 8.0 / kPi;
    if (br == 0) {
        double a2 = a * a, b2 = b * b;
        double s1 = a + b;
        double s3 = (a2 + b2) * s1;
        double s4 = b2 * b2 + b2 * b * a + b2 * a2 + b * a2 * a + a2 * a2;
        return c * bma * (0.5 * s1 - 1.5 * s3 + 1.2 * s4);
    }
    if (br == 1) {
        double pa = 1.0 - a, pb = 1.0 - b;
        double pa2 = pa * pa, pb2 = pb * pb;
        double t3 = (pa2 + pb2) * (pa + pb);
        double t4 = pa2 * pa2 + pa2 * pa * pb + pa2 * pb2 + pa * pb2 * pb + pb2 * pb2;
        return c * bma * (0.5 * t3 - 0.4 * t4);
    }
    return 0.0;
}

// psi(b) - psi(a) for 0 <= a <= b (bma = b - a, formed by the caller without
// cancellation): the part of [a, b] on each polynomial branch ([0, 1/2],
// (1/2, 1]; psi is flat past 1), each by its factored difference.  Both
// branch terms are formed without data-dependent control flow, so the
// quadrature nodes of one piece evaluate side by side.
__device__ __forceinline__ double psi_range(double a, double b, double bma)
{
    const bool a0 = a <= 0.5, a1 = a <= 1.0, b0 = b <= 0.5, b1 = b <= 1.0;
    // branch 0 holds [a, min(b, 1/2)] when a <= 1/2
    const double hi0 = b0 ? b : 0.5;
    const double p0 = psi_piece(0, a, hi0, b0 ? bma : 0.5 - a);
    // branch 1 holds [max(a, 1/2), min(b, 1)] when a <= 1 and b > 1/2
    const double lo1 = a0 ? 0.5 : a, hi1 = b1 ? b : 1.0;
    const double p1 = psi_piece(1, lo1, hi1, (!a0 && b1) ? bma : hi1 - lo1);
    return (a0 ? p0 : 0.0) + ((a1 && !b0) ? p1 : 0.0);
}

// Overlap H(delta, eta) = h_b^3 g for the cubic spline (Appendix D):
//   H = (2 pi / eta^3) int_0^1 ds s^2 w(s) F(s),
//   F(s) = eta^2/(delta s) [psi((s+delta)/eta) - psi(|s-delta|/eta)].
// Between consecutive breakpoints (where s, |s - delta|/eta or (s + delta)/eta
// crosses a branch edge of w or psi) the integrand s w(s) (eta^2/delta)
// [psi(b) - psi(a)] is one polynomial of degree 9 in s (8 for delta = 0), so
// 5-point Gauss-Legendre on each piece is exact up to rounding.
__device__ double overlap_H_exact(double delta, double eta)
{
    if (delta >= 1.0 + eta) return 0.0;
    // 5-point Gauss-Legendre: nodes 0, +-gx[1], +-gx[2] with weights gw[0..2]
    const double gx[3] = {0.0, 0.5384693101056830910, 0.9061798459386639928};
    const double gw[3] = {0.5688888888888888889, 0.4786286704993664680, 0.2369268850561890875};
    // breakpoints of the integrand inside (0, 1), clamped to [0, 1] (those outside give
    // empty pieces), sorted by Batcher's odd-even merge network in registers
    double bp[10] = {0.0, 0.5, delta, delta - 0.5 * eta, delta + 0.5 * eta, delta - eta, delta + eta,
                     0.5 * eta - delta, eta - delta, 1.0};
#pragma unroll
    for (int k = 1; k < 9; ++k) bp[k] = fmin(fmax(bp[k], 0.0), 1.0);
    constexpr int kNet[19][2] = {{1, 2}, {3, 4}, {5, 6}, {7, 8}, {1, 3}, {2, 4}, {5, 7}, {6, 8}, {2, 3}, {6, 7},
                                 {1, 5}, {2, 6}, {3, 7}, {4, 8}, {3, 5}, {4, 6}, {2, 3}, {4, 5}, {6, 7}};
#pragma unroll
    for (int k = 0; k < 19; ++k) {
        const double x = bp[kNet[k][0]], y = bp[kNet[k][1]];
        bp[kNet[k][0]] = fmin(x, y);
        bp[kNet[k][1]] = fmax(x, y);
    }
    // s^2 w(s) F(s) = s w(s) (eta^2/delta) [psi(b) - psi(a)]: one factor s cancels, and the
    // two quotients are formed once per pair, so the nodes take no division
    const double ie = 1.0 / eta, c_ed = delta > 0.0 ? eta * eta / delta : 0.0;
    double acc = 0.0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double lo = bp[k], hi = bp[k + 1];
        if (!(hi > lo)) continue;
        double half = 0.5 * (hi - lo), mid = 0.5 * (hi + lo), piece = 0.0;
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const double s = mid + half * (q < 2 ? -gx[2 - q] : gx[q - 2]);
            const double wq = q < 2 ? gw[2 - q] : gw[q - 2];
            double sF;
            if (delta == 0.0) {
                sF = 2.0 * s * kernel_w(s * ie);
            } else {
                const double a = fabs(s - delta) * ie, b = (s + delta) * ie, bma = 2.0 * fmin(s, delta) * ie;
                sF = c_ed * psi_range(a, b, bma);
            }
            piece += wq * s * kernel_w(s) * sF;
        }
        acc += half * piece;
    }
    return 2.0 * kPi * acc / (eta * eta * eta);
}

// ---------------------------------------------------------------------------
// Overlap for the binary32 path (Appendix D tabulates the overlap; here the
// table keeps RELATIVE accuracy over the whole support, down to pairs that
// barely touch).  With h_b >= h_s, eta = h_s/h_b, delta = d/h_b, H = h_b^3 g:
//   shell (h_b - d < h_s: the small kernel crosses the big one's surface):
//     rho = (h_b + h_s - d)/h_s in [0, 2),  H = eta^3 rho^8 QA(rho, eta);
//   core (h_b - d >= h_s: the small kernel lies inside the big one):
//     kappa = eta/(1 - delta) in (0, 1],  H = (1 - delta)^3 QB(delta, kappa).
// The envelopes carry how H vanishes at the support edge (as its eighth power
// in the distance to contact) and at the big kernel's surface (as the cube),
// so QA and QB are smooth and bounded (QA in [0.0038, 0.146], QB in
// [0.99, 6.3]).  For rho <= 1/2 the shell overlap has the closed form
//   QA = 512/(pi delta) [1/1120 - (1 + eta) rho/2520 + eta rho^2/6300]
// (one polynomial piece of the Appendix D integral), used for the nodes.
// Each region is a kTabN x kTabN grid of cells on [0,1]^2 (x = rho/2 or
// delta, y = eta or kappa); nodes carry Q and its two first derivatives
// scaled by the cell width; the interpolant is cubic Hermite along x for Q,
// linear along x for the y-derivative and cubic Hermite along y, stored per
// cell as polynomial coefficients in the cell offsets (a, b):
//   Q = P0(a) + P1(a) b + P2(a) b^2 + P3(a) b^3,
// P0, P2, P3 cubic and P1 linear in a, as four float4 (P0, P2, P3, P1) = 64
// bytes, so one lookup reads one aligned 64-byte segment.  Interpolation and
// coefficient rounding stay below 6e-7 of g itself.
constexpr int kTabN = 128;
constexpr int kTabCellsRegion = kTabN * kTabN;
constexpr int kTabCells = 2 * kTabCellsRegion;   // shell cells, then core cells

// 1/x for x > 0 in binary64: binary32 reciprocal and one Newton step
// (relative error ~1e-14; no binary64 division).
__device__ __forceinline__ double rcp64(double x)
{
    double r = double(__builtin_amdgcn_rcpf(float(x)));
    return r * fma(-x, r, 2.0);
}

// g(d; h1, h2) in binary64 from the binary64 squared distance of a pair
// inside the support (d2 < (h1 + h2)^2).  The distance is refined from the
// binary32 root by one Newton step in binary64, so that h_b + h_s - d and
// h_b - d keep their relative accuracy near contact.  The value is returned in
// binary64: near contact it falls far below the binary32 range.
__device__ __forceinline__ double overlap_g_table(const float4* __restrict__ tab, double d2, double h1, double h2)
{
    const double hb = h1 > h2 ? h1 : h2, hs = h1 > h2 ? h2 : h1;
    const float d0f = __builtin_amdgcn_sqrtf(float(d2));
    const double d0 = double(d0f);
    const double d = d0f > 0.f ? fma(d2 - d0 * d0, double(0.5f * __builtin_amdgcn_rcpf(d0f)), d0) : 0.0;
    const double ib = rcp64(hb);
    const double inner = hb - d;             // >= hs in the core
    const bool shell = inner < hs;
    const double num = shell ? (hb + hs) - d : hs;
    const double r = num * rcp64(shell ? hs : inner);   // rho (shell) or kappa (core)
    const double eta = hs * ib;
    const double x = shell ? 0.5 * r : d * ib, y = shell ? eta : r;
    const double fx = fmin(x, 1.0) * double(kTabN), fy = fmin(y, 1.0) * double(kTabN);
    const int i = min(int(fx), kTabN - 1), j = min(int(fy), kTabN - 1);
    // the cell polynomial (smooth, positive, of order one) in binary32: its rounding stays
    // below the table's own error; the envelope and the 1/h_b^3 scale stay in binary64
    const float a = float(fx - double(i)), b = float(fy - double(j));
    const float4* c = tab + 4 * ((shell ? 0 : kTabCellsRegion) + j * kTabN + i);
    const float4 q0 = c[0], q2 = c[1], q3 = c[2], q1 = c[3];
    auto cubic = [a](float4 q) { return fmaf(fmaf(fmaf(q.w, a, q.z), a, q.y), a, q.x); };
    const float p0 = cubic(q0), p2 = cubic(q2), p3 = cubic(q3), p1 = fmaf(q1.y, a, q1.x);
    const double Q = double(fmaf(fmaf(fmaf(p3, b, p2), b, p1), b, p0));
    // both envelopes and a select: one basic block, so the scheduler can overlap the cell loads
    const double r2 = r * r, r4 = r2 * r2, tc = inner * ib;
    const double env = shell ? eta * eta * eta * (r4 * r4) : tc * tc * tc;
    return Q * env * (ib * ib * ib);
}

// The same lookup returning binary32, for the binary32 DM pass, whose P_ij
// are binary32: the distance and the two differences that vanish at contact
// (h_b + h_s - d, h_b - d) are still formed in binary64, everything after
// them in binary32 (rounding below 4e-7 of g).  Overlaps under the binary32
// range (pairs within ~1e-5 h_s of contact) flush to zero, as the binary32
// P_ij built from them would.  The gas pass (binary64 terms) takes the
// binary64 lookup for such pairs (overlap_g_gas), so an owner whose every
// neighbour is that close to contact keeps its relative accuracy.
__device__ __forceinline__ float overlap_g_table32(const float4* __restrict__ tab, double d2, double h1, double h2)
{
    const double hbd = h1 > h2 ? h1 : h2, hsd = h1 > h2 ? h2 : h1;
    const float d0f = __builtin_amdgcn_sqrtf(float(d2));
    const double d0 = double(d0f);
    const double d = d0f > 0.f ? fma(d2 - d0 * d0, double(0.5f * __builtin_amdgcn_rcpf(d0f)), d0) : 0.0;
    const double innerd = hbd - d;
    const bool shell = innerd < hsd;
    const float num = float(shell ? (hbd + hsd) - d : hsd);
    const float hb = float(hbd), hs = float(hsd), inner = float(innerd);
    const float ib = __builtin_amdgcn_rcpf(hb);
    const float r = num * __builtin_amdgcn_rcpf(shell ? hs : inner);   // rho (shell) or kappa (core)
    const float eta = hs * ib;
    const float x = shell ? 0.5f * r : float(d) * ib, y = shell ? eta : r;
    const float fx = fminf(x, 1.f) * float(kTabN), fy = fminf(y, 1.f) * float(kTabN);
    const int i = min(int(fx), kTabN - 1), j = min(int(fy), kTabN - 1);
    const float a = fx - float(i), b = fy - float(j);
    const float4* c = tab + 4 * ((shell ? 0 : kTabCellsRegion) + j * kTabN + i);
    const float4 q0 = c[0], q2 = c[1], q3 = c[2], q1 = c[3];
    auto cubic = [a](float4 q) { return fmaf(fmaf(fmaf(q.w, a, q.z), a, q.y), a, q.x); };
    const float p0 = cubic(q0), p2 = cubic(q2), p3 = cubic(q3), p1 = fmaf(q1.y, a, q1.x);
    const float Q = fmaf(fmaf(fmaf(p3, b, p2), b, p1), b, p0);
    const float r2 = r * r, r4 = r2 * r2, tc = inner * ib;
    const float env = shell ? eta * eta * eta * (r4 * r4) : tc * tc * tc;
    return Q * env * (ib * ib * ib);
}

// For the gas pass (binary64 terms): the binary32 lookup, and the binary64
// one for the rare pair so close to contact that its binary32 value nears
// the bottom of the binary32 range, so every overlap keeps its relative
// accuracy.
__device__ __forceinline__ double overlap_g_gas(const float4* __restrict__ tab, double d2, double h1, double h2)
{
    const float g = overlap_g_table32(tab, d2, h1, h2);
    return g >= 1e-30f ? double(g) : overlap_g_table(tab, d2, h1, h2);
}

template <typename T>
__device__ __forceinline__ T overlap_g_exact(T d, T hi, T hj)
{
    double hb = double(hi > hj ? hi : hj), hs = double(hi > hj ? hj : hi);
    return T(overlap_H_exact(double(d) / hb, hs / hb) / (hb * hb * hb));
}

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon et al., SC'11): per round the products M0*x0 and
// M1*x2 give (hi1^x1^k0, lo1, hi0^x3^k1, lo0); key bumped by the Weyl
// constants between rounds.
struct U4 { uint32_t x, y, z, w; };

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1)
{
    // the key schedule is rebuilt per call (scalar adds): hoisted, its 20 words
    // would occupy scalar registers for a whole pass.  Keys are wave-uniform.
    asm volatile("" : "+s"(k0), "+s"(k1));
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        // one 32x32->64 multiply (v_mad_u64_u32) gives both halves
        const uint64_t p0 = uint64_t(c.x) * 0xD2511F53u, p1 = uint64_t(c.z) * 0xCD9E8D57u;
        const uint32_t lo0 = uint32_t(p0), hi0 = uint32_t(p0 >> 32);
        const uint32_t lo1 = uint32_t(p1), hi1 = uint32_t(p1 >> 32);
        U4 n;
        n.x = hi1 ^ c.y ^ k0;
        n.y = lo1;
        n.z = hi0 ^ c.w ^ k1;
        n.w = lo0;
        c = n;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// 24-bit centred uniform ((r >> 8) + 1/2) 2^-24, exactly representable.
template <typename T>
__device__ __forceinline__ T u24(uint32_t r) { return (T(r >> 8) + T(0.5)) * T(1.0 / 16777216.0); }

// Stream layout shared with every consumer of the random numbers:
// counter = (dm index, gas index, step, tag | box << 8), key = seed.
enum : uint32_t { kTagGasVel = 0u, kTagDir = 1u, kTagDecision = 2u, kTagTilt = 5u };

__device__ __forceinline__ U4 philox_block(uint32_t i, uint32_t j, uint32_t step, uint32_t tag, uint32_t box,
                                           uint32_t k0, uint32_t k1)
{
    U4 c{i, j, step, tag | (box << 8)};
    return philox4x32_10(c, k0, k1);
}

// cos(2 pi u), sin(2 pi u): the gfx950 transcendental unit takes turns.
__device__ __forceinline__ void sincos_turns(float u, float* s, float* c)
{
    *s = __builtin_amdgcn_sinf(u);
    *c = __builtin_amdgcn_cosf(u);
}
__device__ __forceinline__ void sincos_turns(double u, double* s, double* c) { sincospi(2.0 * u, s, c); }

// Binary32 uses the hardware units directly: log2 (within 1 ulp) times ln 2,
// square root and reciprocal (1 ulp).  Their arguments on the binary32 path
// are normal numbers or zero, so the library wrappers' rescaling of
// subnormal arguments is not needed.
__device__ __forceinline__ float log_real(float x) { return __builtin_amdgcn_logf(x) * 0.693147180559945309f; }
__device__ __forceinline__ double log_real(double x) { return log(x); }
__device__ __forceinline__ float sqrt_real(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double sqrt_real(double x) { return sqrt(x); }
__device__ __forceinline__ float rcp_real(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double rcp_real(double x) { return 1.0 / x; }

// Three standard normals by Box-Muller from one Philox block.
template <typename T>
__device__ __forceinline__ void normals3(U4 r, T z[3])
{
    T u0 = u24<T>(r.x), u1 = u24<T>(r.y), u2 = u24<T>(r.z), u3 = u24<T>(r.w);
    T r0 = sqrt_real(T(-2) * log_real(u0)), r1 = sqrt_real(T(-2) * log_real(u2));
    T s, c, s2, c2;
    sincos_turns(u1, &s, &c);
    sincos_turns(u3, &s2, &c2);
    z[0] = r0 * c;
    z[1] = r0 * s;
    z[2] = r1 * c2;
}

// ---------------------------------------------------------------------------
// Anisotropic scattering (Sec. 2.2-2.3: dsigma/dOmega = sigma(v) p(Omega)).
// cos theta of the Henyey-Greenstein law p(c) = (1 - g^2) / (2 (1 + g^2 - 2 g c)^{3/2})
// (mean g) from a uniform u by its inverse CDF, and sin theta.  With t = 2u - 1
// the inverse c = (1 + g^2 - s^2) / (2g), s = (1 - g^2) / (1 - g + 2 g u),
// expands to (2t + g (t^2 + 3) + 2 g^2 t + g^3 (t^2 - 1)) / (2 (1 + g t)^2), free
// of the cancellation at small g (g = 0 gives t); and 1 - c^2 factors into
// 4 (1 - g^2)^2 u (1 - u) (1 - g + g u) (1 + g u) / (1 + g t)^4, so sin theta
// keeps its relative accuracy where c is within rounding of +-1.
template <typename T>
__device__ __forceinline__ void hg_angle(T g, T u, T* ct, T* st)
{
    const T t = T(2) * u - T(1), d = T(1) + g * t;
    const T c = (T(2) * t + g * (t * t + T(3)) + T(2) * g * g * t + g * g * g * (t * t - T(1))) / (T(2) * d * d);
    *ct = c < T(-1) ? T(-1) : (c > T(1) ? T(1) : c);
    const T p = u * (T(1) - u) * (T(1) - g + g * u) * (T(1) + g * u);
    *st = T(2) * (T(1) - g * g) * sqrt_real(p > T(0) ? p : T(0)) / (d * d);
}

// Orthonormal e1, e2 with (e1, e2, n) right-handed for a unit n (the
// branch-free construction of Duff et al., J. Comput. Graph. Tech. 6(1), 2017).
template <typename T>
__device__ __forceinline__ void orthonormal_frame(const T n[3], T e1[3], T e2[3])
{
    const T sg = n[2] >= T(0) ? T(1) : T(-1);
    const T a = T(-1) / (sg + n[2]);
    const T b = n[0] * n[1] * a;
    e1[0] = T(1) + sg * n[0] * n[0] * a; e1[1] = sg * b; e1[2] = -sg * n[0];
    e2[0] = b; e2[1] = sg + n[1] * n[1] * a; e2[2] = -n[1];
}

// ---------------------------------------------------------------------------
// Rate functions (Appendix B): for sigma-bar = sigma0 (v/c)^n,
//   A = alpha_n/3 vs^{n+1} 1F1(-(n+1)/2, 5/2, -x),
//   B = alpha_n   vs^{n+3} 1F1(-(n+3)/2, 3/2, -x),  x = w^2/(2 vs^2).
// Here FA, FB are the two 1F1 values.  Large x: erf/exp closed forms of the
// 1F1 for integer n; x < 1: their Taylor series (the closed forms cancel).
template <int N>
struct RateCoef {
    static constexpr int kTerms = 24;
    double ca[kTerms], cb[kTerms];
    constexpr RateCoef() : ca(), cb()
    {
        double a1 = -(N + 1) * 0.5, b1 = 2.5, a2 = -(N + 3) * 0.5, b2 = 1.5;
        double t1 = 1.0, t2 = 1.0;
        for (int k = 0; k < kTerms; ++k) {
            ca[k] = t1;
            cb[k] = t2;
            t1 *= -(a1 + k) / ((b1 + k) * (k + 1));
            t2 *= -(a2 + k) / ((b2 + k) * (k + 1));
        }
    }
};

// Taylor terms for x < 1: binary64 keeps 22; binary32 keeps the fewest whose
// tail (the series alternate) stays below 3e-8 of the value at x = 1.
template <typename T> struct RealTraits;
template <> struct RealTraits<float> {
    template <int N> static constexpr int taylor() { return N == -4 ? 11 : (N == -2 ? 9 : 8); }
};
template <> struct RealTraits<double> {
    template <int N> static constexpr int taylor() { return 22; }
};

__device__ __forceinline__ float erf_real(float x) { return erff(x); }

// erf(t) for t >= 1 in binary32, given e = e^{-t^2}: erf = 1 - e R(t) with
// R(t) = e^{t^2} erfc(t), an entire function, as a degree-12 polynomial in
// t - 2.75 (weighted least-squares fit for relative error on [1, 4.5]; Horner
// in binary32 keeps R within 1.5e-7).  Past t = 4.5, e R < 2^-28 and R(4.5)
// stands in.  Sharing e with the caller saves erf its own exponential.
__device__ __forceinline__ float erf_ge1(float t, float e)
{
    constexpr float c[13] = {1.936620921e-01f, -6.323760748e-02f, 1.975860447e-02f, -5.934607703e-03f,
                             1.719569904e-03f, -4.814862041e-04f, 1.311259839e-04f, -3.548420500e-05f,
                             9.050128938e-06f, -1.834100885e-06f, 4.788607271e-07f, -2.315289720e-07f,
                             5.124300273e-08f};
    const float z = fminf(t, 4.5f) - 2.75f;
    float R = c[12];
#pragma unroll
    for (int k = 11; k >= 0; --k) R = fmaf(R, z, c[k]);
    return fmaf(-e, R, 1.0f);
}
__device__ __forceinline__ double erf_real(double x) { return erf(x); }
__device__ __forceinline__ float exp_neg(float x) { return __expf(-x); }
__device__ __forceinline__ double exp_neg(double x) { return exp(-x); }

template <int N, typename T>
__device__ __forceinline__ void rate_1f1(T x, T* FA, T* FB)
{
    constexpr RateCoef<N> C{};
    if (x < T(1)) {
        constexpr int K = RealTraits<T>::template taylor<N>();
        T fa = T(C.ca[K - 1]), fb = T(C.cb[K - 1]);
#pragma unroll
        for (int k = K - 2; k >= 0; --k) {
            fa = fa * x + T(C.ca[k]);
            fb = fb * x + T(C.cb[k]);
        }
        *FA = fa;
        *FB = fb;
        return;
    }
    T t, r, it;
    if constexpr (sizeof(T) == 4) {
        it = __builtin_amdgcn_rsqf(x);   // x >= 1 here
        t = x * it;
        r = it * it;
    } else {
        t = sqrt_real(x);
        r = T(1) / x;
        it = T(1) / t;
    }
    const T ex = exp_neg(x);
    T E;
    if constexpr (sizeof(T) == 4) E = erf_ge1(t, ex);
    else E = erf_real(t);
    T spE = T(kSqrtPi) * E;
    if constexpr (N == 0) {
        *FA = T(3.0 / 32.0) * (spE * (T(4) * x + T(4) - r) * it + T(2) * (T(2) + r) * ex);
        *FB = (spE * ((T(4) * x + T(12)) * x + T(3)) * it + T(2) * (T(2) * x + T(5)) * ex) * T(1.0 / 16.0);
    } else if constexpr (N == -2) {
        *FA = T(0.75) * ex * r + T(0.75) * spE * it - T(0.375) * spE * r * it;
        *FB = T(0.5) * spE * t + T(0.5) * ex + T(0.25) * spE * it;
    } else if constexpr (N == -4) {
        *FA = T(-1.5) * ex * r + T(0.75) * spE * r * it;
        *FB = T(0.5) * spE * it;
    } else if constexpr (N == 2) {
        *FA = (spE * (((T(8) * x + T(36)) * x + T(18)) * x - T(3)) * it + T(2) * ((T(4) * x + T(16)) * x + T(3)) * ex) *
              (r * T(1.0 / 64.0));
        *FB = (spE * (((T(8) * x + T(60)) * x + T(90)) * x + T(15)) * it + T(2) * ((T(4) * x + T(28)) * x + T(33)) * ex) *
              T(1.0 / 96.0);
    }
}

// Rate integrals by quadrature (for any momentum-transfer cross section;
// used here for sigma-bar = sigma0 (v/c)^n).  With s = u/vs and x = w/vs,
// integrating eq. scrA / scrB over directions of u about w gives
//   A / vs^{n+1} = sqrt(2/pi) (1/x) int_0^inf s^{4+n} e^{-(s^2+x^2)/2} j(s x) ds,
//   B / vs^{n+3} = sqrt(2/pi)       int_0^inf s^{5+n} e^{-(s^2+x^2)/2} sinh(s x)/(s x) ds,
// j(k) = cosh k / k - sinh k / k^2.  The Gaussian factors are formed as
// e^{-(s -+ x)^2/2} (no overflow) and small k uses the Taylor series of j(k)/k
// and sinh(k)/k.  K-node Gauss-Legendre on [max(0, x - hw), max(x + hw, bmin)]
// (hw = 8.5, bmin = 11 reach 1e-10 at K = 32; hw = 5.5, bmin = 7 reach 1e-3
// at K = 12).  Returns the values divided by alpha_n/3 and alpha_n, i.e. in
// the same normalisation as the 1F1 forms of rate_1f1.
template <int N> struct Pow {
    template <typename T> __device__ static __forceinline__ T of(T s)
    {
        if constexpr (N == 0) return T(1);
        else if constexpr (N > 0) return s * Pow<N - 1>::of(s);
        else return T(1) / Pow<-N>::of(s);
    }
};

template <typename T> struct QuadTraits;
template <> struct QuadTraits<float> { static constexpr float kSmall = 0.5f; };
template <> struct QuadTraits<double> { static constexpr double kSmall = 0.1; };

template <int N, typename Real>
__device__ __forceinline__ void rate_quad(Real x, const Real* __restrict__ gx, const Real* __restrict__ gw, int K,
                                          Real inv_alpha, Real hw, Real bmin, Real* FA, Real* FB)
{
    const Real a = x > hw ? x - hw : Real(0);
    const Real b = x + hw > bmin ? x + hw : bmin;
    const Real mid = Real(0.5) * (a + b), half = Real(0.5) * (b - a);
    Real accA = 0, accB = 0;
    for (int q = 0; q < K; ++q) {
        const Real s = mid + half * gx[q];
        const Real k = s * x, k2 = k * k;
        Real jx, es;
        if (k < QuadTraits<Real>::kSmall) {
            const Real e0 = exp_neg(Real(0.5) * (s * s + x * x));
            jx = e0 * s * (Real(1.0 / 3.0) + k2 * (Real(1.0 / 30.0) + k2 * (Real(1.0 / 840.0) + k2 * Real(1.0 / 45360.0))));
            es = e0 * (Real(1) + k2 * (Real(1.0 / 6.0) + k2 * (Real(1.0 / 120.0) + k2 * (Real(1.0 / 5040.0) + k2 * Real(1.0 / 362880.0)))));
        } else {
            const Real g1 = exp_neg(Real(0.5) * (s - x) * (s - x)), g2 = exp_neg(Real(0.5) * (s + x) * (s + x));
            const Real c = Real(0.5) * (g1 + g2), sh = Real(0.5) * (g1 - g2), ik = rcp_real(k);
            jx = (c - sh * ik) * ik * rcp_real(x);
            es = sh * ik;
        }
        const Real p4 = Pow<4 + N>::of(s);
        accA += gw[q] * p4 * jx;
        accB += gw[q] * p4 * s * es;
    }
    const Real c0 = Real(0.79788456080286535588) * half;   // sqrt(2/pi)
    *FA = c0 * accA * Real(3) * inv_alpha;
    *FB = c0 * accB * inv_alpha;
}

// v^{n+1} for the scattering probability P = K g v^{n+1} dt.
template <int N, typename T>
__device__ __forceinline__ T pow_np1(T v)
{
    if constexpr (N == 0) return v;
    else if constexpr (N == -2) return rcp_real(v);
    else if constexpr (N == -4) { T iv = rcp_real(v); return iv * iv * iv; }
    else if constexpr (N == 2) return v * v * v;
    else return T(0);
}

}  // namespace dmb
