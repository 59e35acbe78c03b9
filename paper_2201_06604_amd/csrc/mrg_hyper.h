// mrg_hyper.h -- one contingency-table entry by inversion of its conditional
// hypergeometric distribution (Section 4), host and device.
//
// Definition (the one the oracle evaluates): x in [lo, hi] with weights
// w(lo) = 1, w(x+1) = w(x) * ((K-x)(n-x)) / ((x+1)(N'-K-n+x+1)) in double
// precision (exact integer products, one rounded multiply, one rounded
// divide); the entry is the smallest x with u*W <= w(lo)+...+w(x), sums
// ascending.  Weights above 2^600 and the running sum are scaled by 2^-600
// (exact), and the search compares u*W with the running sum at W's scale:
// the mantissas of the same operations on an unbounded exponent range.
//
// Two shortcuts give the same bits with less work:
//  * The first pass (W) stops once the ratio has dropped below 1 (the
//    weights only decrease from there: num/den <= 1 - 2^-40, so even after
//    two roundings each weight is below the previous one) and the next weight
//    is below W * 2^-54 (under half an ulp of W): every later addition rounds
//    back to W.
//  * The first pass records NCK checkpoints (partial sum before x_c, w(x_c),
//    scale count) at x_c = lo + c*step; partial sums never decrease, so the
//    search starts at the last checkpoint whose partial sum is below u*W and
//    runs the same operations from there.
#pragma once

#include <stdint.h>

#include <cmath>

#ifndef MRG_HD
#if defined(__HIPCC__)
#define MRG_HD __host__ __device__
#else
#define MRG_HD
#endif
#endif

namespace mrg355 {

constexpr double kHyperBig = 0x1p600;
constexpr int kHyperScaleExp = 600;

// Checkpoint storage: element c of a lane at s[c*stride], w[c*stride],
// r[c*stride] (LDS on the device, a plain array on the host).
struct HyperCk {
    double* s;
    double* w;
    int* r;
    int stride;
};

// The integer products of the ratio are formed in fp64: with every total at
// most 2^20 (the callers' bound) each factor is an integer below 2^21 and each
// product below 2^42, so the fp64 products are exact and equal the integer
// products converted to double.
template <int NCK>
MRG_HD inline int hyper_invert_ck(double u, int64_t Np, int64_t K, int64_t n, HyperCk ck) {
    int64_t lo = n - (Np - K);
    if (lo < 0) lo = 0;
    const int64_t hi = n < K ? n : K;
    if (hi <= lo) return static_cast<int>(lo);
    const int64_t step = (hi - lo + NCK) / NCK;  // ceil(span / NCK), span = hi - lo + 1
    const double Kd = static_cast<double>(K), nd = static_cast<double>(n);
    const double rest = static_cast<double>(Np - K - n + 1);  // N' - K - n + 1
    int64_t next = lo;
    int nck = 0;
    double W = 0.0, w = 1.0;
    int scales = 0;
    double xd = static_cast<double>(lo);
    for (int64_t x = lo; x <= hi; ++x, xd += 1.0) {
        if (x == next) {
            ck.s[nck * ck.stride] = W;
            ck.w[nck * ck.stride] = w;
            ck.r[nck * ck.stride] = scales;
            ++nck;
            next += step;
        }
        W += w;
        if (x < hi) {
            const double num = (Kd - xd) * (nd - xd);
            const double den = (xd + 1.0) * (rest + xd);
            w = w * num / den;
            if (w > kHyperBig) {
                w = ldexp(w, -kHyperScaleExp);
                W = ldexp(W, -kHyperScaleExp);
                ++scales;
            }
            if (num < den && w * 0x1p54 < W) break;
        }
    }
    const double target = u * W;
    int c = 0;
    for (int k = 1; k < nck; ++k) {
        if (ldexp(ck.s[k * ck.stride], -kHyperScaleExp * (scales - ck.r[k * ck.stride])) < target) c = k;
        else break;
    }
    double s = ck.s[c * ck.stride];
    w = ck.w[c * ck.stride];
    int done = ck.r[c * ck.stride];
    xd = static_cast<double>(lo + c * step);
    for (int64_t x = lo + c * step; x <= hi; ++x, xd += 1.0) {
        s += w;
        if (target <= ldexp(s, -kHyperScaleExp * (scales - done))) return static_cast<int>(x);
        const double num = (Kd - xd) * (nd - xd);
        const double den = (xd + 1.0) * (rest + xd);
        w = w * num / den;
        if (w > kHyperBig) {
            w = ldexp(w, -kHyperScaleExp);
            s = ldexp(s, -kHyperScaleExp);
            ++done;
        }
    }
    return static_cast<int>(hi);
}

}  // namespace mrg355
