// mrg_math.h -- MRG32k3a constants and exact modular matrix arithmetic for the
// product library (host code and compile-time device tables).
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
// Reduction uses the special form m = 2^32 - c: 2^32 = c (mod m), so a 64-bit
// value h*2^32 + l folds to h*c + l.  Everything here is constexpr so that the
// device jump tables are computed by the compiler.
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

struct Mat3 {
    uint32_t a[9];
};

// x mod (2^32 - c) for any 64-bit x, 1 <= c < 2^15.
MRG_HD constexpr uint32_t fold64(uint64_t x, uint32_t c) {
    x = (x >> 32) * c + (x & 0xffffffffull);  // < 2^47 + 2^32
    x = (x >> 32) * c + (x & 0xffffffffull);  // < 2^32 + 2^30 + c
    x = (x >> 32) * c + (x & 0xffffffffull);  // < 2^32
    uint32_t r = static_cast<uint32_t>(x);
    uint32_t m = 0u - c;
    return r >= m ? r - m : r;
}

MRG_HD constexpr uint32_t mulmod(uint32_t a, uint32_t b, uint32_t c) {
    return fold64(static_cast<uint64_t>(a) * b, c);
}

MRG_HD constexpr uint32_t addmod(uint32_t a, uint32_t b, uint32_t c) {
    return fold64(static_cast<uint64_t>(a) + b, c);
}

MRG_HD constexpr Mat3 identity() { return Mat3{{1, 0, 0, 0, 1, 0, 0, 0, 1}}; }

// One-step matrices on (x[n-3], x[n-2], x[n-1]) -> (x[n-2], x[n-1], x[n]).
MRG_HD constexpr Mat3 step_matrix(int comp) {
    return comp == 0 ? Mat3{{0, 1, 0, 0, 0, 1, kM1 - kA13N, kA12, 0}}
                     : Mat3{{0, 1, 0, 0, 0, 1, kM2 - kA23N, 0, kA21}};
}

MRG_HD constexpr uint32_t comp_c(int comp) { return comp == 0 ? kC1 : kC2; }

MRG_HD constexpr Mat3 matmul(const Mat3& A, const Mat3& B, uint32_t c) {
    Mat3 C{};
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            uint32_t acc = 0;
            for (int t = 0; t < 3; ++t) acc = addmod(acc, mulmod(A.a[r * 3 + t], B.a[t * 3 + k], c), c);
            C.a[r * 3 + k] = acc;
        }
    return C;
}

// A^(2^k) by k squarings.
MRG_HD constexpr Mat3 pow2k(Mat3 A, int k, uint32_t c) {
    for (int i = 0; i < k; ++i) A = matmul(A, A, c);
    return A;
}

// A^e for a 64-bit exponent.
MRG_HD constexpr Mat3 matpow(Mat3 A, uint64_t e, uint32_t c) {
    Mat3 R = identity();
    while (e) {
        if (e & 1) R = matmul(R, A, c);
        A = matmul(A, A, c);
        e >>= 1;
    }
    return R;
}

// v <- M v (mod 2^32 - c) on one component.
MRG_HD constexpr void matvec(const Mat3& M, uint32_t v[3], uint32_t c) {
    uint32_t t[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r) {
        uint64_t acc = 0;
        for (int k = 0; k < 3; ++k) acc += mulmod(M.a[r * 3 + k], v[k], c);
        t[r] = fold64(acc, c);
    }
    v[0] = t[0];
    v[1] = t[1];
    v[2] = t[2];
}

// Per-bit jump tables: step_pow2[j][b] = A_j^(2^b), stream_pow2[j][b] =
// A_j^(2^(127+b)) (b < 64), substream[j] = A_j^(2^76).
struct JumpTables {
    Mat3 step_pow2[2][64];
    Mat3 stream_pow2[2][64];
    Mat3 substream[2];
};

MRG_HD constexpr JumpTables make_jump_tables() {
    JumpTables T{};
    for (int j = 0; j < 2; ++j) {
        uint32_t c = comp_c(j);
        Mat3 A = step_matrix(j);
        for (int b = 0; b < 64; ++b) {
            T.step_pow2[j][b] = A;
            A = matmul(A, A, c);
        }
        // continue squaring from A^(2^64) up to A^(2^127)
        for (int b = 64; b < kStreamLog2; ++b) A = matmul(A, A, c);
        for (int b = 0; b < 64; ++b) {
            T.stream_pow2[j][b] = A;
            A = matmul(A, A, c);
        }
        T.substream[j] = pow2k(step_matrix(j), kSubstreamLog2, c);
    }
    return T;
}

}  // namespace mrg355
