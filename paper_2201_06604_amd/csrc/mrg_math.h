// mrg_math.h -- constants of the two generators and exact modular matrix
// arithmetic for the product library (host code and compile-time device
// tables).
//
// The generator is MRG32k3a (L'Ecuyer 1999; named by the clrng paper in
// Sections 1, 2 and 6):
//   x1[n] = ( 1403580 x1[n-2] -  810728 x1[n-3]) mod m1,  m1 = 2^32 - 209
//   x2[n] = (  527612 x2[n-1] - 1370589 x2[n-3]) mod m2,  m2 = 2^32 - 22853
//   z[n]  = (x1[n] - x2[n]) mod m1, mapped to [1, m1]   (0 becomes m1)
// Streams are Z = 2^127 steps apart and substreams 2^76 (Section 2.1 cuts the
// period into pieces of length Z; RngStreams fixes Z and the substream
// spacing for MRG32k3a).  Jump-ahead multiplies the per-component state
// vector (x[n-3], x[n-2], x[n-1]) by a power of the one-step matrix.
//
// The second generator is MRG31k3p (L'Ecuyer and Touzin 2000), the one the
// clrng paper itself uses (Section 2):
//   x1[n] = (2^22 x1[n-2] + (2^7 + 1) x1[n-3]) mod p1,   p1 = 2^31 - 1
//   x2[n] = (2^15 x2[n-1] + (2^15 + 1) x2[n-3]) mod p2,  p2 = 2^31 - 21069
//   z[n]  = (x1[n] - x2[n]) mod p1 in [1, p1], u = z / 2^31
// with streams 2^134 apart (Section 2.1) and substreams 2^72 apart.  Its
// states are kept newest-first, (x[n-1], x[n-2], x[n-3]) per component, the
// order of the stream table printed in Section 2.1, so its matrices act on
// that order.
//
// Reduction uses the special form m = 2^B - c (B = 32 or 31): 2^B = c (mod m),
// so a 64-bit value h*2^B + l folds to h*c + l.  Everything here is constexpr
// so that the device jump tables are computed by the compiler.
#pragma once

#include <stdint.h>

#ifndef MRG_HD
#if defined(__HIPCC__)
#define MRG_HD __host__ __device__
#else
#define MRG_HD
#endif
#endif

namespace mrg355 {

constexpr uint32_t kC1 = 209u;
constexpr uint32_t kC2 = 22853u;
constexpr uint32_t kM1 = 0u - kC1;  // 4294967087
constexpr uint32_t kM2 = 0u - kC2;  // 4294944443
constexpr uint32_t kA12 = 1403580u;
constexpr uint32_t kA13N = 810728u;
constexpr uint32_t kA21 = 527612u;
constexpr uint32_t kA23N = 1370589u;
// 1/(m1+1) rounded to double: the scale of Section 2.2 (the integer in
// [1, m1] times one constant).
constexpr double kNorm = 1.0 / 4294967088.0;
constexpr int kStreamLog2 = 127;
constexpr int kSubstreamLog2 = 76;

constexpr uint32_t kQ1 = 1u;
constexpr uint32_t kQ2 = 21069u;
constexpr uint32_t kP1 = 0x80000000u - kQ1;  // 2147483647
constexpr uint32_t kP2 = 0x80000000u - kQ2;  // 2147462579
constexpr uint32_t kB12 = 1u << 22;          // multiplies x1[n-2]
constexpr uint32_t kB13 = (1u << 7) + 1u;    // multiplies x1[n-3]
constexpr uint32_t kB21 = 1u << 15;          // multiplies x2[n-1]
constexpr uint32_t kB23 = (1u << 15) + 1u;   // multiplies x2[n-3]
constexpr double kNorm31 = 1.0 / 2147483648.0;  // 2^-31, exact
constexpr int kStreamLog2_31 = 134;
constexpr int kSubstreamLog2_31 = 72;

// Generator ids used inside the library (the ABI's ids minus one).
enum Generator { kGen32k3a = 0, kGen31k3p = 1 };

struct Mat3 {
    uint32_t a[9];
};

// x mod (2^B - c) for any 64-bit x, B = 32 or 31, 1 <= c < 2^15.  Each fold
// maps h*2^B + l to h*c + l.  B = 32: three folds leave x < 2^32 (the bounds
// below); B = 31: four folds leave x < 2^31.  Then x < 2m and one
// conditional subtraction finishes.
template <int B = 32>
MRG_HD constexpr uint32_t fold64(uint64_t x, uint32_t c) {
    constexpr uint64_t mask = (static_cast<uint64_t>(1) << B) - 1;
    if constexpr (B == 32) {
        x = (x >> 32) * c + (x & mask);  // < 2^47 + 2^32
        x = (x >> 32) * c + (x & mask);  // < 2^32 + 2^30 + c
        x = (x >> 32) * c + (x & mask);  // < 2^32
    } else {
        x = (x >> 31) * c + (x & mask);  // < 2^48 + 2^31
        x = (x >> 31) * c + (x & mask);  // < 2^32 + 2^31
        x = (x >> 31) * c + (x & mask);  // < 2^31 + 2c
        x = (x >> 31) * c + (x & mask);  // < 2^31
    }
    const uint64_t m = (static_cast<uint64_t>(1) << B) - c;
    return static_cast<uint32_t>(x >= m ? x - m : x);
}

template <int B = 32>
MRG_HD constexpr uint32_t mulmod(uint32_t a, uint32_t b, uint32_t c) {
    return fold64<B>(static_cast<uint64_t>(a) * b, c);
}

template <int B = 32>
MRG_HD constexpr uint32_t addmod(uint32_t a, uint32_t b, uint32_t c) {
    return fold64<B>(static_cast<uint64_t>(a) + b, c);
}

MRG_HD constexpr Mat3 identity() { return Mat3{{1, 0, 0, 0, 1, 0, 0, 0, 1}}; }

// MRG32k3a one-step matrices on (x[n-3], x[n-2], x[n-1]) -> (x[n-2], x[n-1], x[n]).
MRG_HD constexpr Mat3 step_matrix(int comp) {
    return comp == 0 ? Mat3{{0, 1, 0, 0, 0, 1, kM1 - kA13N, kA12, 0}}
                     : Mat3{{0, 1, 0, 0, 0, 1, kM2 - kA23N, 0, kA21}};
}

// MRG31k3p one-step matrices on (x[n-1], x[n-2], x[n-3]) -> (x[n], x[n-1], x[n-2]).
MRG_HD constexpr Mat3 step_matrix31(int comp) {
    return comp == 0 ? Mat3{{0, kB12, kB13, 1, 0, 0, 0, 1, 0}} : Mat3{{kB21, 0, kB23, 1, 0, 0, 0, 1, 0}};
}

MRG_HD constexpr uint32_t comp_c(int comp) { return comp == 0 ? kC1 : kC2; }
MRG_HD constexpr uint32_t comp_c31(int comp) { return comp == 0 ? kQ1 : kQ2; }

template <int B = 32>
MRG_HD constexpr Mat3 matmul(const Mat3& A, const Mat3& Bm, uint32_t c) {
    Mat3 C{};
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            uint32_t acc = 0;
            for (int t = 0; t < 3; ++t)
                acc = addmod<B>(acc, mulmod<B>(A.a[r * 3 + t], Bm.a[t * 3 + k], c), c);
            C.a[r * 3 + k] = acc;
        }
    return C;
}

// A^(2^k) by k squarings.
template <int B = 32>
MRG_HD constexpr Mat3 pow2k(Mat3 A, int k, uint32_t c) {
    for (int i = 0; i < k; ++i) A = matmul<B>(A, A, c);
    return A;
}

// A^e for a 64-bit exponent.
template <int B = 32>
MRG_HD constexpr Mat3 matpow(Mat3 A, uint64_t e, uint32_t c) {
    Mat3 R = identity();
    while (e) {
        if (e & 1) R = matmul<B>(R, A, c);
        A = matmul<B>(A, A, c);
        e >>= 1;
    }
    return R;
}

// v <- M v (mod 2^B - c) on one component.
template <int B = 32>
MRG_HD constexpr void matvec(const Mat3& M, uint32_t v[3], uint32_t c) {
    uint32_t t[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r) {
        uint64_t acc = 0;
        for (int k = 0; k < 3; ++k) acc += mulmod<B>(M.a[r * 3 + k], v[k], c);
        t[r] = fold64<B>(acc, c);
    }
    v[0] = t[0];
    v[1] = t[1];
    v[2] = t[2];
}

// v <- M v (mod m) in fp64, exactly, for m < 2^32, entries of M and v below
// m.  Each word of v is split into 16-bit halves, so every product is below
// 2^48 and each row's two 3-term sums below 2^50; a sum A is reduced as
// A - rint(A/m) m (one FMA, exact: the nearest quotient is off by at most
// one and the result stays below m in magnitude), the halves recombine as
// a*2^16 + B < 2^51, and a final floor step maps into [0, m).
// The same integers as matvec<B>(), with floating-point multiply-adds.
MRG_HD inline double f64_mod_near(double a, double m, double inv_m) {
    return __builtin_fma(-__builtin_rint(a * inv_m), m, a);
}

MRG_HD inline void matvec_f64(const double M[9], double v[3], double m, double inv_m) {
    double hi[3], lo[3], t[3];
    for (int k = 0; k < 3; ++k) {
        hi[k] = __builtin_floor(v[k] * (1.0 / 65536.0));
        lo[k] = __builtin_fma(-hi[k], 65536.0, v[k]);
    }
    for (int r = 0; r < 3; ++r) {
        const double a = __builtin_fma(M[r * 3 + 2], hi[2], __builtin_fma(M[r * 3 + 1], hi[1], M[r * 3] * hi[0]));
        const double b = __builtin_fma(M[r * 3 + 2], lo[2], __builtin_fma(M[r * 3 + 1], lo[1], M[r * 3] * lo[0]));
        const double c = f64_mod_near(__builtin_fma(f64_mod_near(a, m, inv_m), 65536.0, b), m, inv_m);
        t[r] = __builtin_fma(-__builtin_floor(c * inv_m), m, c);  // [0, m)
    }
    v[0] = t[0];
    v[1] = t[1];
    v[2] = t[2];
}

// Per-bit jump tables: step_pow2[j][b] = A_j^(2^b), stream_pow2[j][b] =
// A_j^(2^(Z+b)) (b < 64; Z = 127 or 134), substream[j] = A_j^(2^76 or 2^72).
struct JumpTables {
    Mat3 step_pow2[2][64];
    Mat3 stream_pow2[2][64];
    Mat3 substream[2];
};

template <int G>
MRG_HD constexpr JumpTables make_jump_tables() {
    constexpr int B = G == kGen32k3a ? 32 : 31;
    constexpr int zlog = G == kGen32k3a ? kStreamLog2 : kStreamLog2_31;
    constexpr int slog = G == kGen32k3a ? kSubstreamLog2 : kSubstreamLog2_31;
    JumpTables T{};
    for (int j = 0; j < 2; ++j) {
        const uint32_t c = G == kGen32k3a ? comp_c(j) : comp_c31(j);
        const Mat3 A1 = G == kGen32k3a ? step_matrix(j) : step_matrix31(j);
        Mat3 A = A1;
        for (int b = 0; b < 64; ++b) {
            T.step_pow2[j][b] = A;
            A = matmul<B>(A, A, c);
        }
        // continue squaring from A^(2^64) up to A^(2^Z)
        for (int b = 64; b < zlog; ++b) A = matmul<B>(A, A, c);
        for (int b = 0; b < 64; ++b) {
            T.stream_pow2[j][b] = A;
            A = matmul<B>(A, A, c);
        }
        T.substream[j] = pow2k<B>(A1, slog, c);
    }
    return T;
}

// Stream jumps by base-64 digits: digit[d][j][v] = J^(v 64^d) for component
// j (J = the jump between neighbouring streams, A^(2^127) or A^(2^134)), so
// J^i for a stream index i < 2^36 is the product of at most six entries, one
// per nonzero base-64 digit of i (powers of one matrix commute).
constexpr int kStreamDigits = 6;
struct StreamDigits {
    Mat3 digit[kStreamDigits][2][64];
};

template <int G>
MRG_HD constexpr StreamDigits make_stream_digits(const JumpTables& T) {
    constexpr int B = G == kGen32k3a ? 32 : 31;
    StreamDigits D{};
    for (int j = 0; j < 2; ++j) {
        const uint32_t c = G == kGen32k3a ? comp_c(j) : comp_c31(j);
        for (int d = 0; d < kStreamDigits; ++d) {
            const Mat3& base = T.stream_pow2[j][6 * d];  // J^(64^d)
            Mat3 P = identity();
            for (int v = 0; v < 64; ++v) {
                D.digit[d][j][v] = P;
                P = matmul<B>(P, base, c);
            }
        }
    }
    return D;
}

// Step jumps by base-64 digits, for the fp64 engine: digit[d][j][v] =
// A_j^(v 64^d) with entries as doubles, so A^e for any e < 2^64 is the product
// of at most eleven entries, one per nonzero base-64 digit of e, each applied
// with matvec_f64 (a chunk start inside a stream: e = offset + j * chunk).
constexpr int kStepDigits = 11;
struct StepDigitsF64 {
    double m[kStepDigits][2][64][9];
};

template <int G>
MRG_HD constexpr StepDigitsF64 make_step_digits_f64(const JumpTables& T) {
    constexpr int B = G == kGen32k3a ? 32 : 31;
    StepDigitsF64 D{};
    for (int j = 0; j < 2; ++j) {
        const uint32_t c = G == kGen32k3a ? comp_c(j) : comp_c31(j);
        for (int d = 0; d < kStepDigits; ++d) {
            const int bit = 6 * d;
            const Mat3 base = bit < 64 ? T.step_pow2[j][bit] : identity();  // A^(64^d)
            Mat3 P = identity();
            for (int v = 0; v < 64; ++v) {
                for (int k = 0; k < 9; ++k) D.m[d][j][v][k] = static_cast<double>(P.a[k]);
                P = matmul<B>(P, base, c);
            }
        }
    }
    return D;
}

}  // namespace mrg355
