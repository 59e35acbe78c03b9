// mrg_engine.h -- the exact generator steps on gfx950 (device code, included
// by the kernel sources).  MRG32k3a in two interchangeable arithmetic forms:
//
//   IntEngine  32x32->64 multiply-adds, reduced with 2^32 = c (mod 2^32 - c)
//   F64Engine  the same integers held exactly in fp64: every product is below
//              2^53 and each remainder p - q*m is one exact FMA
//
// Both give identical integers z in [1, m1].  MRG31k3p (Engine31) uses 32-bit
// rotations for its power-of-two multipliers modulo the Mersenne prime p1 and
// one 64-bit fold modulo p2.
//
// Every engine keeps each component as a ring of three registers holding
// (x[n-3], x[n-2], x[n-1]); a step overwrites x[n-3] with x[n], so a 3-step
// cycle needs no register moves.  Both recurrences read x1[n-2], x1[n-3],
// x2[n-1] and x2[n-3], so the ring logic is shared.
#pragma once

#include <hip/hip_runtime.h>

#include "mrg_logtab.h"
#include "mrg_sincostab.h"
#include "mrg_math.h"

namespace mrg355 {

// -------------------------------------------------------- integer engine
// p < 2^54 -> p mod m1.  p = h*2^32 + l with h < 2^22; 2^32 = 209 (mod m1).
__device__ __forceinline__ uint32_t fold_m1(uint64_t p) {
    uint32_t h = static_cast<uint32_t>(p >> 32), l = static_cast<uint32_t>(p);
    uint64_t t = static_cast<uint64_t>(__umul24(h, kC1)) + l;          // < 2^32 + 2^30
    uint32_t r = static_cast<uint32_t>(t) + static_cast<uint32_t>(t >> 32) * kC1;
    return min(r, r - kM1);                                             // r < 2^32 < 2 m1
}

// p < 2^54 -> p mod m2.  h < 2^21, 2^32 = 22853 (mod m2).
__device__ __forceinline__ uint32_t fold_m2(uint64_t p) {
    uint32_t h = static_cast<uint32_t>(p >> 32), l = static_cast<uint32_t>(p);
    uint64_t t = static_cast<uint64_t>(h) * kC2 + l;                   // < 2^36 + 2^32
    uint32_t h2 = static_cast<uint32_t>(t >> 32), l2 = static_cast<uint32_t>(t);
    uint64_t t2 = static_cast<uint64_t>(__umul24(h2, kC2)) + l2;       // < 2^32 + 2^19
    uint32_t r = static_cast<uint32_t>(t2) + static_cast<uint32_t>(t2 >> 32) * kC2;
    return min(r, r - kM2);
}

struct IntEngine {
    uint32_t a0, a1, a2, b0, b1, b2;  // (x1[n-3], x1[n-2], x1[n-1]), (x2[...])

    __device__ __forceinline__ void load(const uint32_t x[6]) {
        a0 = x[0]; a1 = x[1]; a2 = x[2]; b0 = x[3]; b1 = x[4]; b2 = x[5];
    }
    __device__ __forceinline__ void save(uint32_t x[6]) const {
        x[0] = a0; x[1] = a1; x[2] = a2; x[3] = b0; x[4] = b1; x[5] = b2;
    }
    // New x1 from (x1[n-2], x1[n-3]) replaces x1[n-3]; new x2 from (x2[n-1],
    // x2[n-3]) replaces x2[n-3]; returns z in [1, m1].
    static __device__ __forceinline__ uint32_t kernel(uint32_t& o1, uint32_t m2_1, uint32_t& o2,
                                                      uint32_t n1_2) {
        uint64_t p1 = static_cast<uint64_t>(kA12) * m2_1 + static_cast<uint64_t>(kA13N) * (kM1 - o1);
        uint64_t p2 = static_cast<uint64_t>(kA21) * n1_2 + static_cast<uint64_t>(kA23N) * (kM2 - o2);
        uint32_t x1 = fold_m1(p1), x2 = fold_m2(p2);
        o1 = x1;
        o2 = x2;
        return x1 > x2 ? x1 - x2 : x1 - x2 + kM1;
    }
    // Phase-P step of a 3-step cycle: the ring of registers rotates by naming,
    // so no moves are needed.
    template <int P>
    __device__ __forceinline__ uint32_t step() {
        if (P == 0) return kernel(a0, a1, b0, b2);
        if (P == 1) return kernel(a1, a2, b1, b0);
        return kernel(a2, a0, b2, b1);
    }
    __device__ __forceinline__ uint32_t step_rot() {
        uint32_t z = kernel(a0, a1, b0, b2);
        uint32_t t = a0; a0 = a1; a1 = a2; a2 = t;
        t = b0; b0 = b1; b1 = b2; b2 = t;
        return z;
    }
};

// ------------------------------------------------------- MRG31k3p engine
// 2^k x mod (2^31 - 1) for x < 2^31 - 1: a 31-bit rotation (2^31 = 1).  The
// result is below 2^31 - 1 because x is.
template <int K>
__device__ __forceinline__ uint32_t rot31(uint32_t x) {
    return ((x << K) & kP1) | (x >> (31 - K));
}

// a + b mod m for a, b < m < 2^31: one conditional subtraction (min picks the
// reduced value; a + b - m wraps above it when a + b < m).
__device__ __forceinline__ uint32_t add_mod31(uint32_t a, uint32_t b, uint32_t m) {
    const uint32_t s = a + b;
    return min(s, s - m);
}

struct Engine31 {
    uint32_t a0, a1, a2, b0, b1, b2;  // (x1[n-3], x1[n-2], x1[n-1]), (x2[...])

    // The stored state is newest-first: (x1[n-1], x1[n-2], x1[n-3], x2[...]).
    __device__ __forceinline__ void load(const uint32_t x[6]) {
        a0 = x[2]; a1 = x[1]; a2 = x[0]; b0 = x[5]; b1 = x[4]; b2 = x[3];
    }
    __device__ __forceinline__ void save(uint32_t x[6]) const {
        x[0] = a2; x[1] = a1; x[2] = a0; x[3] = b2; x[4] = b1; x[5] = b0;
    }
    // o1 = x1[n-3] (becomes x1[n]), m2_1 = x1[n-2], o2 = x2[n-3] (becomes
    // x2[n]), n1_2 = x2[n-1]; returns z in [1, p1].
    static __device__ __forceinline__ uint32_t kernel(uint32_t& o1, uint32_t m2_1, uint32_t& o2,
                                                      uint32_t n1_2) {
        // x1[n] = 2^22 x1[n-2] + 2^7 x1[n-3] + x1[n-3]  (mod p1)
        const uint32_t x1 = add_mod31(add_mod31(rot31<22>(m2_1), rot31<7>(o1), kP1), o1, kP1);
        // x2[n] = 2^15 (x2[n-1] + x2[n-3]) + x2[n-3]  (mod p2), p < 2^47 + 2^31
        const uint64_t p = (static_cast<uint64_t>(n1_2 + o2) << 15) + o2;
        const uint32_t h = static_cast<uint32_t>(p >> 31), l = static_cast<uint32_t>(p) & 0x7fffffffu;
        const uint32_t t = __umul24(h, kQ2) + l;                      // h < 2^17: t < 2^32
        const uint32_t t2 = (t >> 31) * kQ2 + (t & 0x7fffffffu);      // < 2^31 + q2 < 2 p2
        const uint32_t x2 = min(t2, t2 - kP2);
        o1 = x1;
        o2 = x2;
        return x1 > x2 ? x1 - x2 : x1 - x2 + kP1;
    }
    template <int P>
    __device__ __forceinline__ uint32_t step() {
        if (P == 0) return kernel(a0, a1, b0, b2);
        if (P == 1) return kernel(a1, a2, b1, b0);
        return kernel(a2, a0, b2, b1);
    }
    __device__ __forceinline__ uint32_t step_rot() {
        uint32_t z = kernel(a0, a1, b0, b2);
        uint32_t t = a0; a0 = a1; a1 = a2; a2 = t;
        t = b0; b0 = b1; b1 = b2; b2 = t;
        return z;
    }
};

// ------------------------------------------------------------ fp64 engine
constexpr double kM1d = static_cast<double>(kM1);
constexpr double kM2d = static_cast<double>(kM2);
constexpr double kInvM1 = 1.0 / kM1d;
constexpr double kInvM2 = 1.0 / kM2d;

// p an integer with |p| < 2^53 -> an integer r = p (mod m) with
// |r| <= m/2 + 4, exactly: q is the nearest quotient (off by at most one),
// and p - q*m is exact in one FMA.
__device__ __forceinline__ double f64_rem(double p, double m, double inv_m) {
    double q = __builtin_rint(p * inv_m);
    return __builtin_fma(-q, m, p);
}

// |r| <= m/2 + 4 -> r mod m in [0, m): floor(r/m) is -1 or 0.
__device__ __forceinline__ double f64_canon(double r, double m, double inv_m) {
    double t = __builtin_floor(r * inv_m);
    return __builtin_fma(-t, m, r);
}

// Component 1 is carried as any residue with |x| <= m1/2 + 4 (its value only
// matters mod m1); component 2 is kept in [0, m2) because z uses its value.
// Products stay below 2^53 in magnitude either way, so every FMA is exact.
struct F64Engine {
    double a0, a1, a2, b0, b1, b2;

    __device__ __forceinline__ void load(const uint32_t x[6]) {
        a0 = x[0]; a1 = x[1]; a2 = x[2]; b0 = x[3]; b1 = x[4]; b2 = x[5];
    }
    __device__ __forceinline__ void save(uint32_t x[6]) const {
        x[0] = static_cast<uint32_t>(f64_canon(a0, kM1d, kInvM1));
        x[1] = static_cast<uint32_t>(f64_canon(a1, kM1d, kInvM1));
        x[2] = static_cast<uint32_t>(f64_canon(a2, kM1d, kInvM1));
        x[3] = static_cast<uint32_t>(b0); x[4] = static_cast<uint32_t>(b1);
        x[5] = static_cast<uint32_t>(b2);
    }
    static __device__ __forceinline__ double kernel(double& o1, double m2_1, double& o2, double n1_2) {
        double p1 = __builtin_fma(static_cast<double>(kA12), m2_1, -(static_cast<double>(kA13N) * o1));
        double p2 = __builtin_fma(static_cast<double>(kA21), n1_2, -(static_cast<double>(kA23N) * o2));
        double x1 = f64_rem(p1, kM1d, kInvM1);
        double x2 = f64_canon(f64_rem(p2, kM2d, kInvM2), kM2d, kInvM2);
        o1 = x1;
        o2 = x2;
        // z = d mod m1 in [1, m1], d = x1 - x2 in [-(1.5 m1 + 4), m1/2 + 4]:
        // t = floor((d-1)/m1) in {-2, -1, 0}.  Near a multiple of m1 the
        // quotient differs from it by at least 1/m1, far above the rounding
        // of the FMA, so t is exact.
        double d = x1 - x2;
        double t = __builtin_floor(__builtin_fma(d, kInvM1, -kInvM1));
        return __builtin_fma(-t, kM1d, d);
    }
    template <int P>
    __device__ __forceinline__ double step() {
        if (P == 0) return kernel(a0, a1, b0, b2);
        if (P == 1) return kernel(a1, a2, b1, b0);
        return kernel(a2, a0, b2, b1);
    }
    __device__ __forceinline__ double step_rot() {
        double z = kernel(a0, a1, b0, b2);
        double t = a0; a0 = a1; a1 = a2; a2 = t;
        t = b0; b0 = b1; b1 = b2; b2 = t;
        return z;
    }
};

// ------------------------------------------------------------- transforms
// sin(pi t) and cos(pi t) for t = 2u in (0, 2) (the Box-Muller angle).
// n = rint(2t), r = t - n/2 in [-1/4, 1/4] (exact: t and n/2 are within a
// factor of two, or n = 0); sin(pi r) and cos(pi r) by their Taylor series in
// r^2 with pi folded into the coefficients (sine through r^17, cosine through
// r^16: the next terms are below 2^-58 at |r| = 1/4); the quadrant n mod 4
// swaps and negates.  mrg_transform_accuracy compares both results with the
// HIP library's sincospi over any range of generator outputs.
__device__ __forceinline__ void sincospi_unit_series(double t, double* sp, double* cp) {
    const double n = __builtin_rint(t + t);
    const double r = __builtin_fma(n, -0.5, t);
    const double z = r * r;
    double ps = 7.952054001475513e-07;
    ps = __builtin_fma(ps, z, -2.1915353447830217e-05);
    ps = __builtin_fma(ps, z, 0.00046630280576761255);
    ps = __builtin_fma(ps, z, -0.0073704309457143504);
    ps = __builtin_fma(ps, z, 0.08214588661112823);
    ps = __builtin_fma(ps, z, -0.5992645293207921);
    ps = __builtin_fma(ps, z, 2.5501640398773455);
    ps = __builtin_fma(ps, z, -5.16771278004997);
    ps = __builtin_fma(ps, z, 3.141592653589793);
    const double sn = r * ps;
    double pc = 4.303069587032947e-06;
    pc = __builtin_fma(pc, z, -0.0001046381049248457);
    pc = __builtin_fma(pc, z, 0.0019295743094039231);
    pc = __builtin_fma(pc, z, -0.02580689139001406);
    pc = __builtin_fma(pc, z, 0.2353306303588932);
    pc = __builtin_fma(pc, z, -1.3352627688545895);
    pc = __builtin_fma(pc, z, 4.0587121264167685);
    pc = __builtin_fma(pc, z, -4.934802200544679);
    const double cs = __builtin_fma(pc, z, 1.0);
    // quadrant q = n mod 4 (n in 0..4): odd q swaps sine and cosine; the sine
    // is negative for q = 2, 3 (bit 1 of n) and the cosine for q = 1, 2 (bit 1
    // of n + 1), applied as a flip of the sign bit in the high word
    const uint32_t ni = static_cast<uint32_t>(static_cast<int>(n));
    const double s1 = (ni & 1u) ? cs : sn;
    const double c1 = (ni & 1u) ? sn : cs;
    const uint32_t sgn_s = (ni << 30) & 0x80000000u;
    const uint32_t sgn_c = ((ni + 1u) << 30) & 0x80000000u;
    *sp = __hiloint2double(__double2hiint(s1) ^ static_cast<int>(sgn_s), __double2loint(s1));
    *cp = __hiloint2double(__double2hiint(c1) ^ static_cast<int>(sgn_c), __double2loint(c1));
}


// sqrt(x) for the Box-Muller radius argument x = -2 log(u1) in [2^-32, 47]:
// never zero, subnormal or non-finite, so the range scaling and special
// cases of a general square root are left out.  Goldschmidt's iteration from
// the hardware reciprocal square root y ~ 1/sqrt(x): g ~ sqrt(x) and
// h ~ 1/(2 sqrt(x)) are refined together once, then one Newton correction
// g += h (x - g^2) with an exact residual (FMA).  mrg_transform_accuracy
// compares it with the HIP library's sqrt on the radius argument of any range
// of generator outputs: bit-identical over every output of both generators
// (a second correction changed no result).
__device__ __forceinline__ double sqrt_radius(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    double g = x * y;
    double h = 0.5 * y;
    const double r = __builtin_fma(-h, g, 0.5);
    g = __builtin_fma(g, r, g);
    h = __builtin_fma(h, r, h);
    const double d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, h, g);
}

// log(u) for the generators' uniforms, u in [2^-33, 1): never zero,
// subnormal, negative or non-finite, so no special cases.  u = m 2^k with m
// in [sqrt(1/2), sqrt(2)); f = m - 1 (exact); s = f / d with d = 2 + f;
// log(m) = 2 atanh(s) = 2s + 2s (s^2/3 + s^4/5 + ... + s^18/19) (|s| <=
// 0.1716, so the next term is below 2^-55 relative); log(u) = k ln2 + log(m)
// with ln2 split so that k * ln2_hi is exact.  d = 2 + f is rounded (f can
// carry a bit below d's last place), so s has up to about one ulp of relative
// error whatever the division does; the quotient itself uses the hardware
// reciprocal (relative error below 5e-8 on these divisors), one Newton step
// and one residual correction q += (f - q d) y, which leave a quotient of the
// rounded d accurate far below an ulp.  mrg_transform_accuracy compares the
// result with the HIP library's log over any range of generator outputs.
// SCALE (1, -1, 2 or -2) multiplies the result: it is folded into the last
// three steps' constants, and scaling by a power of two commutes with
// rounding, so log_unit<SCALE>(u) is bit for bit SCALE * log_unit(u).
template <int SCALE = 1>
__device__ __forceinline__ double log_unit_series(double u) {
    static_assert(SCALE == 1 || SCALE == -1 || SCALE == 2 || SCALE == -2, "power-of-two scale");
    int k = __builtin_amdgcn_frexp_exp(u);          // u = mant * 2^k, mant in [1/2, 1)
    double m = __builtin_amdgcn_frexp_mant(u);
    // below sqrt(1/2) the mantissa is doubled (an exponent step, exact) and k
    // lowered: one integer select and an ldexp rather than a 64-bit select
    const int lo = m < 0.70710678118654752440 ? 1 : 0;
    m = __builtin_amdgcn_ldexp(m, lo);
    k -= lo;
    const double f = m - 1.0;
    const double d = 2.0 + f;
    double y = __builtin_amdgcn_rcp(d);
    const double e = __builtin_fma(-d, y, 1.0);
    y = __builtin_fma(e, y, y);
    double q = f * y;
    q = __builtin_fma(__builtin_fma(-q, d, f), y, q);  // s = f / d
    const double z = q * q;
    double r = 1.0 / 19.0;
    r = __builtin_fma(r, z, 1.0 / 17.0);
    r = __builtin_fma(r, z, 1.0 / 15.0);
    r = __builtin_fma(r, z, 1.0 / 13.0);
    r = __builtin_fma(r, z, 1.0 / 11.0);
    r = __builtin_fma(r, z, 1.0 / 9.0);
    r = __builtin_fma(r, z, 1.0 / 7.0);
    r = __builtin_fma(r, z, 1.0 / 5.0);
    r = __builtin_fma(r, z, 1.0 / 3.0);
    r = r * z;
    const double s2 = q * (2.0 * SCALE);
    const double log_m = __builtin_fma(s2, r, s2);
    const double kd = static_cast<double>(k);
    constexpr double kLn2Hi = 6.93147180369123816490e-01;  // ln 2 to 32 bits: k * hi exact for |k| < 2^20
    constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - hi
    return __builtin_fma(kd, kLn2Hi * SCALE, __builtin_fma(kd, kLn2Lo * SCALE, log_m));
}

// The tables of log_unit (mrg_logtab.h) and sincospi_unit (mrg_sincostab.h)
// in LDS: every kernel whose code evaluates the fp64 transforms stages them
// once per block with stage_tables() (all threads, then a barrier) before any
// call.
static __constant__ LogTable g_logtab = kLogTable;
static __constant__ SinCosTable g_sincostab = kSinCosTable;

__device__ __forceinline__ double* log_table_lds() {
    __shared__ double tab[kLogTabN * 3];
    return tab;
}

__device__ __forceinline__ double* sincos_table_lds() {
    __shared__ double tab[kSinCosTabN * 4];
    return tab;
}

// Every wave writes both tables whole (the same values): loops of fixed trip
// count over the wave's lanes, with no dependence on the block size (a loop
// bounded by threadIdx and blockDim made the compiler treat later row addresses
// as divergent).
__device__ __forceinline__ void stage_tables() {
    double* t = log_table_lds();
    double* c = sincos_table_lds();
    const int lane = static_cast<int>(threadIdx.x & 63);
#pragma unroll
    for (int k = 0; k < kLogTabN * 3 / 64; ++k) {
        const int i = lane + 64 * k;
        t[i] = g_logtab.e[i / 3][i % 3];
    }
#pragma unroll
    for (int k = 0; k < (kSinCosTabN * 4 + 63) / 64; ++k) {
        const int i = lane + 64 * k;
        if (i < kSinCosTabN * 4) c[i] = g_sincostab.e[i / 4][i % 4];
    }
    __syncthreads();
}

// sin(pi t) and cos(pi t) for t = 2u in (0, 2) (the Box-Muller angle), by
// table: j = rint(64 t) and d = t - j/64 (exact: t and j/64 are within a
// factor of two, or j = 0; |d| <= 1/128); with s_j = sin(pi j/64) and
// c_j = cos(pi j/64) from the table as hi + lo,
// sin(pi t) = s_j + (s_j (cos(pi d) - 1) + c_j sin(pi d))
// and cos(pi t) = c_j + (c_j (cos(pi d) - 1) - s_j sin(pi d)), where
// sin(pi d) runs through d^7 and cos(pi d) - 1 through d^6 (the next terms
// are below 2^-60 of sin(pi d) and 3.3e-18 in absolute value at |d| = 1/128:
// even where cos(pi t) is smallest beside a nonzero c_j, j = 31 or 33, that is
// under 2^-57 of the result).  On the axes (j a multiple
// of 32) the table holds exact zeros and ones, so results near the zeros of
// sin and cos keep their relative accuracy.  mrg_transform_accuracy compares
// both results with the HIP library's sincospi over any range of generator
// outputs.
__device__ __forceinline__ void sincospi_unit(double t, double* sp, double* cp) {
    const double jd = __builtin_rint(t * 64.0);
    const double d = __builtin_fma(jd, -1.0 / 64.0, t);
    const double* e = sincos_table_lds() + 4 * static_cast<int>(jd);
    const double z = d * d;
    double ps = -0.5992645293207921;  // -pi^7/7!
    ps = __builtin_fma(ps, z, 2.5501640398773455);  // pi^5/5!
    ps = __builtin_fma(ps, z, -5.16771278004997);   // -pi^3/3!
    ps = __builtin_fma(ps, z, 3.141592653589793);   // pi
    const double sd = d * ps;
    double pc = -1.3352627688545895;                // -pi^6/6!
    pc = __builtin_fma(pc, z, 4.0587121264167685);  // pi^4/4!
    pc = __builtin_fma(pc, z, -4.934802200544679);  // -pi^2/2!
    const double cm1 = z * pc;
    const double sh = e[0], sl = e[1], ch = e[2], cl = e[3];
    *sp = sh + __builtin_fma(sh, cm1, __builtin_fma(ch, sd, sl));
    *cp = ch + __builtin_fma(ch, cm1, __builtin_fma(-sh, sd, cl));
}

// log(u) for the generators' uniforms, u in [2^-33, 1), by table: u = m 2^k
// with m in [1/2, 1); the top 9 fraction bits of m pick an interval of width
// 1/1024 whose entry holds R, a multiple of 2^-9 near 1/m (R = 1 on the last
// interval), and -log(R) = hi + lo.  t = m R - 1 is exact (|t| < 2^-9, a
// multiple of 2^-62), log(m) = -log(R) + log1p(t) with log1p(t) = t + t^2 P(t)
// through t^6 (the next term, t^7/7, is below 2^-65: under 2^-55 of any
// result outside the last interval, where |log u| >= 2^-10, and below 2^-54
// of t on the last one), and k ln2 + hi is exact (hi a multiple of 2^-40,
// ln2_hi of 2^-32, |k| <= 33).  Near u = 1 (k = 0, R = 1) the result is
// log1p(t) alone, accurate relative to its own size.
// SCALE (1, -1, 2 or -2) multiplies the result exactly.
// mrg_transform_accuracy compares it with the HIP library's log over any
// range of generator outputs.
template <int SCALE = 1>
__device__ __forceinline__ double log_unit(double u) {
    static_assert(SCALE == 1 || SCALE == -1 || SCALE == 2 || SCALE == -2, "power-of-two scale");
    const int k = __builtin_amdgcn_frexp_exp(u);
    const double m = __builtin_amdgcn_frexp_mant(u);  // [1/2, 1)
    static_assert(kLogTabN == 512, "the index takes the top 9 fraction bits of m");
    const uint32_t j = (static_cast<uint32_t>(__double2hiint(m)) >> 11) & (kLogTabN - 1);
    const double* e = log_table_lds() + 3 * j;
    const double t = __builtin_fma(m, e[0], -1.0);
    double p = -1.0 / 6.0;
    p = __builtin_fma(p, t, 1.0 / 5.0);
    p = __builtin_fma(p, t, -1.0 / 4.0);
    p = __builtin_fma(p, t, 1.0 / 3.0);
    p = __builtin_fma(p, t, -1.0 / 2.0);
    const double q = (t * t) * p;
    const double kd = static_cast<double>(k);
    constexpr double kLn2Hi = 6.93147180369123816490e-01;  // ln 2 to 32 bits: k * hi exact
    constexpr double kLn2Lo = 1.90821492927058770002e-10;  // ln 2 - hi
    const double a = __builtin_fma(kd, kLn2Hi, e[1]);
    const double lo = __builtin_fma(kd, kLn2Lo, e[2]);
    return (a + (t + (q + lo))) * SCALE;
}

// ----------------------------------------------- transforms for fp32 output
// A normal or exponential draw stored as a float needs its value to about
// 1e-7 relative, not to the last bit of a double, so these evaluate the same
// formulas with shorter series and no refinement of the hardware estimates.
// Their results are rounded to float.  Each function's relative error
// (bounds below, checked over every generator output by
// mrg_transform_accuracy) stays under 2e-7.  The largest error of a stored
// float is then under 4e-7 of max(|value|, 1), against the 1e-6 fp32
// tolerance.

// log(u) by log_unit's table (staged in LDS by the calling kernel): t = m R - 1
// exact, |t| < 2^-9, and log1p(t) through t^3 (the next term, t^4/4 < 2^-38,
// is below 2^-28 of any result outside the last interval, where
// |log u| >= 2^-10, and below 2^-29 of t on the last one); -log R's low part
// (below 2^-40) and the low bits of ln 2 are left out (below 2^-30 of the
// result).  Near u = 1 (k = 0, R = 1) the result is log1p(t) alone, accurate
// relative to its own size.
template <int SCALE = 1>
__device__ __forceinline__ double log_unit_f32out(double u) {
    static_assert(SCALE == 1 || SCALE == -1 || SCALE == 2 || SCALE == -2, "power-of-two scale");
    const int k = __builtin_amdgcn_frexp_exp(u);
    const double m = __builtin_amdgcn_frexp_mant(u);  // [1/2, 1)
    const uint32_t j = (static_cast<uint32_t>(__double2hiint(m)) >> 11) & (kLogTabN - 1);
    const double* e = log_table_lds() + 3 * j;
    const double t = __builtin_fma(m, e[0], -1.0);
    const double q = (t * t) * __builtin_fma(t, 1.0 / 3.0, -0.5);
    constexpr double kLn2 = 6.93147180559945286227e-01;
    return (__builtin_fma(static_cast<double>(k), kLn2, e[1]) + (t + q)) * SCALE;
}

// sqrt(x) for the radius argument, x in [2^-32, 47]: the hardware reciprocal
// square root and one Newton correction of g = x y (relative error of the
// order of the estimate's square, far below 1e-7).
__device__ __forceinline__ double sqrt_radius_f32out(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double g = x * y;
    const double d = __builtin_fma(-g, g, x);
    return __builtin_fma(d, 0.5 * y, g);
}

// sin(pi t), cos(pi t) by sincospi_unit's table (staged in LDS by the calling
// kernel, the high parts only): d = t - j/64, |d| <= 1/128, sin(pi d) through
// d^3 (next term below 3e-9 of it) and cos(pi d) - 1 through d^2 (next term
// below 1.5e-8 in absolute value; beside the zero of cos(pi t) it is scaled
// by |c_j| <= 0.05, under 4e-8 of the result there).  On the axes the table
// holds exact zeros and ones, so results near the zeros of sin and cos keep
// their relative accuracy.
__device__ __forceinline__ void sincospi_unit_f32out(double t, double* sp, double* cp) {
    const double jd = __builtin_rint(t * 64.0);
    const double d = __builtin_fma(jd, -1.0 / 64.0, t);
    const double* e = sincos_table_lds() + 4 * static_cast<int>(jd);
    const double z = d * d;
    const double sd = d * __builtin_fma(z, -5.16771278004997, 3.141592653589793);  // pi d - (pi d)^3/6
    const double cm1 = z * -4.934802200544679;                                     // -(pi d)^2/2
    const double sh = e[0], ch = e[2];
    *sp = __builtin_fma(ch, sd, __builtin_fma(sh, cm1, sh));
    *cp = __builtin_fma(-sh, sd, __builtin_fma(ch, cm1, ch));
}

__device__ __forceinline__ double to_f64(uint32_t z) { return static_cast<double>(z); }
__device__ __forceinline__ double to_f64(double z) { return z; }
__device__ __forceinline__ uint32_t to_u32(uint32_t z) { return z; }
__device__ __forceinline__ uint32_t to_u32(double z) { return static_cast<uint32_t>(z); }

}  // namespace mrg355
