// mrg_kernels.hip -- gfx950 kernels of the multi-stream MRG32k3a generator.
//
// Hot path (generate): one work-item owns one stream for one chunk of its
// draws.  The 6-word state lives in VGPRs for the whole chunk; the recurrence
// is exact integer arithmetic mod m1 / m2 (MRG32k3a, L'Ecuyer 1999); the
// uniform, Box-Muller (Algorithm 1) and inverse-transform exponential
// (Section 3.2) outputs are formed in registers and written straight to HBM.
//
// Output layout: draw k of stream s goes to element k*S + s, so the 64 lanes
// of a wave (64 consecutive streams at the same draw index) write one
// contiguous 256/512-byte segment per draw.  A wave owns (64 streams) x (one
// chunk of draw indices); chunk j starts from the stream's current state
// jumped ahead j*chunk steps with per-bit matrix powers read from constant
// memory (the exponent is wave-uniform, so these are scalar loads).  All
// work-items of a stream read its state when they start, so when a stream is
// split over several chunks its state is advanced afterwards by a separate
// small kernel; a stream held by one work-item is written back in place.
//
// Two exact arithmetic forms of the same recurrence:
//   kArithInt  32x32->64 multiply-adds, reduced with 2^32 = c (mod 2^32 - c)
//   kArithF64  the same integers held exactly in fp64: each product and the
//              remainder p - q*m are exact FMAs (all magnitudes < 2^53)
// Both produce identical integers; tests check both against the oracle.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mrg_internal.h"
#include "mrg_math.h"

namespace mrg355 {

__constant__ JumpTables g_tab = make_jump_tables();
static constexpr JumpTables kHostTab = make_jump_tables();

// ------------------------------------------------------------------ jumps
__device__ __forceinline__ void dev_apply(const Mat3& M1, const Mat3& M2, uint32_t x[6]) {
    matvec(M1, x, kC1);
    matvec(M2, x + 3, kC2);
}

// x <- A^e x, e wave-uniform.
__device__ __forceinline__ void dev_jump(uint32_t x[6], uint64_t e) {
    for (int b = 0; e; ++b, e >>= 1)
        if (e & 1) dev_apply(g_tab.step_pow2[0][b], g_tab.step_pow2[1][b], x);
}

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

// ------------------------------------------------------------ fp64 engine
constexpr double kM1d = static_cast<double>(kM1);
constexpr double kM2d = static_cast<double>(kM2);
constexpr double kInvM1 = 1.0 / kM1d;
constexpr double kInvM2 = 1.0 / kM2d;

// p an integer with |p| < 2^53 -> p mod m in [0, m), exactly.
__device__ __forceinline__ double f64_mod(double p, double m, double inv_m) {
    double q = __builtin_rint(p * inv_m);       // nearest quotient (off by <= 1)
    double r = __builtin_fma(-q, m, p);         // exact, |r| <= m/2 + 4
    double t = __builtin_floor(r * inv_m);      // -1 or 0
    return __builtin_fma(-t, m, r);             // exact, in [0, m)
}

struct F64Engine {
    double a0, a1, a2, b0, b1, b2;

    __device__ __forceinline__ void load(const uint32_t x[6]) {
        a0 = x[0]; a1 = x[1]; a2 = x[2]; b0 = x[3]; b1 = x[4]; b2 = x[5];
    }
    __device__ __forceinline__ void save(uint32_t x[6]) const {
        x[0] = static_cast<uint32_t>(a0); x[1] = static_cast<uint32_t>(a1);
        x[2] = static_cast<uint32_t>(a2); x[3] = static_cast<uint32_t>(b0);
        x[4] = static_cast<uint32_t>(b1); x[5] = static_cast<uint32_t>(b2);
    }
    static __device__ __forceinline__ double kernel(double& o1, double m2_1, double& o2, double n1_2) {
        // a12 x - a13n y and a21 x - a23n y are exact: every term < 2^53.
        double p1 = __builtin_fma(static_cast<double>(kA12), m2_1, -(static_cast<double>(kA13N) * o1));
        double p2 = __builtin_fma(static_cast<double>(kA21), n1_2, -(static_cast<double>(kA23N) * o2));
        double x1 = f64_mod(p1, kM1d, kInvM1), x2 = f64_mod(p2, kM2d, kInvM2);
        o1 = x1;
        o2 = x2;
        // z = d if d >= 1 else d + m1, d = x1 - x2 in [-(m2-1), m1-1]:
        // floor((d-1)/m1) is -1 or 0 and is computed exactly enough here.
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
__device__ __forceinline__ double to_f64(uint32_t z) { return static_cast<double>(z); }
__device__ __forceinline__ double to_f64(double z) { return z; }
__device__ __forceinline__ uint32_t to_u32(uint32_t z) { return z; }
__device__ __forceinline__ uint32_t to_u32(double z) { return static_cast<uint32_t>(z); }

// Largest float <= u for u in [2^-126, 1): drop the low 29 mantissa bits
// after rebasing the exponent (1023 -> 127).
__device__ __forceinline__ float f32_rz(double u) {
    uint64_t b = static_cast<uint64_t>(__double_as_longlong(u));
    uint64_t r = b - (static_cast<uint64_t>(896) << 52);
    return __uint_as_float(static_cast<uint32_t>(r >> 29));
}

template <typename T, bool NT>
__device__ __forceinline__ void put(T* p, T v) {
    if (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Store one uniform / raw / exponential draw with value from z.
template <int DIST, int DTYPE, bool NT, typename Z>
__device__ __forceinline__ void emit1(void* row, int lane, Z z, double inv_rate) {
    if (DIST == kRaw) {
        put<uint32_t, NT>(static_cast<uint32_t*>(row) + lane, to_u32(z));
        return;
    }
    double u = to_f64(z) * kNorm;
    double v = u;
    if (DIST == kExponential) v = -log(u) * inv_rate;
    if (DTYPE == kF64) {
        put<double, NT>(static_cast<double*>(row) + lane, v);
    } else {
        float f = DIST == kUniform ? f32_rz(u) : static_cast<float>(v);
        put<float, NT>(static_cast<float*>(row) + lane, f);
    }
}

// Box-Muller pair (Algorithm 1) from two consecutive steps of one stream.
template <typename Z>
__device__ __forceinline__ void box_muller(Z z1, Z z2, double& x, double& y) {
    double u1 = to_f64(z1) * kNorm, u2 = to_f64(z2) * kNorm;
    double r = sqrt(-2.0 * log(u1));
    double s, c;
    sincospi(2.0 * u2, &s, &c);
    x = r * c;
    y = r * s;
}

template <int DTYPE, bool NT>
__device__ __forceinline__ void emit_val(void* row, int lane, double v) {
    if (DTYPE == kF64) put<double, NT>(static_cast<double*>(row) + lane, v);
    else put<float, NT>(static_cast<float*>(row) + lane, static_cast<float>(v));
}

template <int DTYPE>
__device__ __forceinline__ char* advance_row(char* row, uint64_t S) {
    return row + S * (DTYPE == kF64 ? 8 : 4);
}

// ------------------------------------------------------------ generate
template <int DIST, int DTYPE, int ARITH, bool NT>
__global__ void __launch_bounds__(1024) gen_kernel(GenLaunch L) {
    using Engine = typename std::conditional<ARITH == kArithF64, F64Engine, IntEngine>::type;
    constexpr int ESZ = DTYPE == kF64 ? 8 : 4;
    const int lane = threadIdx.x & 63;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t sblk = blockIdx.x * (blockDim.x >> 6) + wave;
    const uint32_t n_sblk = (L.S + 63) >> 6;
    if (sblk >= n_sblk) return;
    const uint32_t s = sblk * 64 + lane;
    if (s >= L.S) return;

    // Work is counted in units: draws, or Box-Muller pairs for normals.
    const uint64_t cnt = L.q + (s < L.r ? 1 : 0);
    const uint64_t cnt_max = L.q + (L.r ? 1 : 0);
    const uint64_t units = DIST == kNormal ? (cnt + 1) / 2 : cnt;
    const uint64_t units_max = DIST == kNormal ? (cnt_max + 1) / 2 : cnt_max;
    const uint64_t full = DIST == kNormal ? L.q / 2 : L.q;  // units every stream completes
    const uint64_t u0 = static_cast<uint64_t>(blockIdx.y) * L.chunk;
    if (u0 >= units) return;
    const uint64_t u1 = min(u0 + L.chunk, units_max);
    constexpr uint64_t kSpu = DIST == kNormal ? 2 : 1;  // steps per unit

    uint32_t* rec = L.streams + static_cast<uint64_t>(s) * 18;
    uint32_t x[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) x[i] = rec[i];
    if (u0) dev_jump(x, u0 * kSpu);
    Engine e;
    e.load(x);

    const double inv_rate = L.param;
    const uint64_t S = L.S;
    const uint64_t kend = max(u0, min(u1, full));
    uint64_t k = u0;
    // Uniform row pointer: first draw of this chunk, first stream of the wave.
    char* row = static_cast<char*>(L.out) + (k * kSpu * S + static_cast<uint64_t>(sblk) * 64) * ESZ;

    if (DIST == kNormal) {
        for (; k + 3 <= kend; k += 3) {
            double x0, y0, x1v, y1v, x2v, y2v;
            auto z0 = e.template step<0>();
            auto z1 = e.template step<1>();
            auto z2 = e.template step<2>();
            auto z3 = e.template step<0>();
            auto z4 = e.template step<1>();
            auto z5 = e.template step<2>();
            box_muller(z0, z1, x0, y0);
            box_muller(z2, z3, x1v, y1v);
            box_muller(z4, z5, x2v, y2v);
            emit_val<DTYPE, NT>(row, lane, x0); row = advance_row<DTYPE>(row, S);
            emit_val<DTYPE, NT>(row, lane, y0); row = advance_row<DTYPE>(row, S);
            emit_val<DTYPE, NT>(row, lane, x1v); row = advance_row<DTYPE>(row, S);
            emit_val<DTYPE, NT>(row, lane, y1v); row = advance_row<DTYPE>(row, S);
            emit_val<DTYPE, NT>(row, lane, x2v); row = advance_row<DTYPE>(row, S);
            emit_val<DTYPE, NT>(row, lane, y2v); row = advance_row<DTYPE>(row, S);
        }
        for (; k < kend; ++k) {
            double xv, yv;
            auto z0 = e.step_rot();
            auto z1 = e.step_rot();
            box_muller(z0, z1, xv, yv);
            emit_val<DTYPE, NT>(row, lane, xv); row = advance_row<DTYPE>(row, S);
            emit_val<DTYPE, NT>(row, lane, yv); row = advance_row<DTYPE>(row, S);
        }
        // Ragged tail (at most one pair): X and Y only where they exist.
        const uint64_t tend = min(u1, units);
        for (; k < tend; ++k) {
            double xv, yv;
            auto z0 = e.step_rot();
            auto z1 = e.step_rot();
            box_muller(z0, z1, xv, yv);
            if (2 * k < cnt) emit_val<DTYPE, NT>(row, lane, xv);
            row = advance_row<DTYPE>(row, S);
            if (2 * k + 1 < cnt) emit_val<DTYPE, NT>(row, lane, yv);
            row = advance_row<DTYPE>(row, S);
        }
    } else {
        for (; k + 3 <= kend; k += 3) {
            auto z0 = e.template step<0>();
            emit1<DIST, DTYPE, NT>(row, lane, z0, inv_rate); row = advance_row<DTYPE>(row, S);
            auto z1 = e.template step<1>();
            emit1<DIST, DTYPE, NT>(row, lane, z1, inv_rate); row = advance_row<DTYPE>(row, S);
            auto z2 = e.template step<2>();
            emit1<DIST, DTYPE, NT>(row, lane, z2, inv_rate); row = advance_row<DTYPE>(row, S);
        }
        for (; k < kend; ++k) {
            auto z = e.step_rot();
            emit1<DIST, DTYPE, NT>(row, lane, z, inv_rate); row = advance_row<DTYPE>(row, S);
        }
        const uint64_t tend = min(u1, units);
        for (; k < tend; ++k) {
            auto z = e.step_rot();
            emit1<DIST, DTYPE, NT>(row, lane, z, inv_rate); row = advance_row<DTYPE>(row, S);
        }
    }

    // A stream owned by a single work-item is written back here; otherwise
    // finalize_kernel advances it after this launch (other chunks of the same
    // stream may not have read it yet).
    if (L.n_chunks == 1) {
        e.save(x);
#pragma unroll
        for (int i = 0; i < 6; ++i) rec[i] = x[i];
    }
}

// cur <- A^(steps consumed) cur for every stream, after a chunked launch:
// cnt_s = q + (s < r) draws; normals consume 2*ceil(cnt_s/2) steps.
__global__ void __launch_bounds__(256) finalize_kernel(uint32_t* streams, uint32_t S, uint64_t q,
                                                       uint32_t r, int normal) {
    uint32_t s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    uint64_t cnt = q + (s < r ? 1 : 0);
    uint64_t steps = normal ? (cnt + 1) / 2 * 2 : cnt;
    uint32_t* rec = streams + static_cast<uint64_t>(s) * 18;
    uint32_t x[6];
#pragma unroll
    for (int w = 0; w < 6; ++w) x[w] = rec[w];
    for (int b = 0; b < 64; ++b)  // uniform loop: table loads stay scalar
        if ((steps >> b) & 1) dev_apply(g_tab.step_pow2[0][b], g_tab.step_pow2[1][b], x);
#pragma unroll
    for (int w = 0; w < 6; ++w) rec[w] = x[w];
}

// ------------------------------------------------------ stream creation
// Stream i = J^i creator with J = A^(2^127): multiply by J^(2^b) for each
// set bit b of i (the per-bit tables are uniform scalar loads).
__global__ void __launch_bounds__(256) create_kernel(uint32_t* out, uint64_t n, uint32_t c0, uint32_t c1,
                                                     uint32_t c2, uint32_t c3, uint32_t c4, uint32_t c5,
                                                     int nbits) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t x[6] = {c0, c1, c2, c3, c4, c5};
    for (int b = 0; b < nbits; ++b)
        if ((i >> b) & 1) dev_apply(g_tab.stream_pow2[0][b], g_tab.stream_pow2[1][b], x);
    uint32_t* rec = out + i * 18;
#pragma unroll
    for (int w = 0; w < 6; ++w) {
        rec[w] = x[w];
        rec[6 + w] = x[w];
        rec[12 + w] = x[w];
    }
}

__global__ void __launch_bounds__(256) reset_kernel(uint32_t* streams, uint64_t n, int kind) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t* rec = streams + i * 18;
    uint32_t x[6];
    if (kind == 0) {  // cur = sub = start
#pragma unroll
        for (int w = 0; w < 6; ++w) x[w] = rec[6 + w];
    } else {
#pragma unroll
        for (int w = 0; w < 6; ++w) x[w] = rec[12 + w];
        if (kind == 2) dev_apply(g_tab.substream[0], g_tab.substream[1], x);
    }
#pragma unroll
    for (int w = 0; w < 6; ++w) {
        rec[w] = x[w];
        rec[12 + w] = x[w];
    }
}

__global__ void __launch_bounds__(256) advance_kernel(uint32_t* streams, uint64_t n, uint64_t steps) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t* rec = streams + i * 18;
    uint32_t x[6];
#pragma unroll
    for (int w = 0; w < 6; ++w) x[w] = rec[w];
    dev_jump(x, steps);
#pragma unroll
    for (int w = 0; w < 6; ++w) rec[w] = x[w];
}

// ------------------------------------------------------------ host side
void host_jump_pow2(uint32_t state[6], uint64_t k, bool stream_tables) {
    for (int b = 0; k; ++b, k >>= 1) {
        if (!(k & 1)) continue;
        const Mat3& A = stream_tables ? kHostTab.stream_pow2[0][b] : kHostTab.step_pow2[0][b];
        const Mat3& B = stream_tables ? kHostTab.stream_pow2[1][b] : kHostTab.step_pow2[1][b];
        matvec(A, state, kC1);
        matvec(B, state + 3, kC2);
    }
}

static unsigned grid1d(uint64_t n, unsigned block) {
    return static_cast<unsigned>((n + block - 1) / block);
}

hipError_t launch_create(uint32_t* out, uint64_t n, const uint32_t c[6], hipStream_t s) {
    int nbits = 0;
    while (nbits < 64 && ((n - 1) >> nbits)) ++nbits;
    hipLaunchKernelGGL(create_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, out, n, c[0], c[1], c[2],
                       c[3], c[4], c[5], nbits);
    return hipGetLastError();
}

hipError_t launch_reset(uint32_t* streams, uint64_t n, int kind, hipStream_t s) {
    hipLaunchKernelGGL(reset_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, streams, n, kind);
    return hipGetLastError();
}

hipError_t launch_advance(uint32_t* streams, uint64_t n, uint64_t steps, hipStream_t s) {
    hipLaunchKernelGGL(advance_kernel, dim3(grid1d(n, 256)), dim3(256), 0, s, streams, n, steps);
    return hipGetLastError();
}

// Automatic launch shape: enough waves to cover the chip several times over
// (256 CUs x 4 SIMDs), chunks of at least 96 units, at most 65535 chunks.
void plan_generate(GenLaunch& L) {
    if (!L.arith) L.arith = kArithInt;
    if (!L.block) L.block = 256;
    const uint64_t cnt_max = L.q + (L.r ? 1 : 0);
    const uint64_t units_max = L.dist == kNormal ? (cnt_max + 1) / 2 : cnt_max;
    const uint64_t n_sblk = (static_cast<uint64_t>(L.S) + 63) / 64;
    if (!L.chunk) {
        const uint64_t target_waves = 16384;
        uint64_t w = (target_waves + n_sblk - 1) / n_sblk;
        uint64_t w_cap = (units_max + 95) / 96;
        if (w > w_cap) w = w_cap;
        if (w < 1) w = 1;
        uint64_t c = (units_max + w - 1) / w;
        c = (c + 2) / 3 * 3;
        L.chunk = static_cast<uint32_t>(c > 0xffffffffull ? 0xffffffffull : (c ? c : 1));
    }
    uint64_t nch = units_max ? (units_max + L.chunk - 1) / L.chunk : 0;
    if (nch > 65535) {
        uint64_t c = (units_max + 65534) / 65535;
        L.chunk = static_cast<uint32_t>(c);
        nch = (units_max + c - 1) / c;
    }
    L.n_chunks = static_cast<uint32_t>(nch);
}

template <int DIST, int DTYPE, int ARITH, bool NT>
static hipError_t launch_t(const GenLaunch& L, hipStream_t s) {
    const unsigned wpb = static_cast<unsigned>(L.block) / 64;
    const uint64_t n_sblk = (static_cast<uint64_t>(L.S) + 63) / 64;
    dim3 grid(static_cast<unsigned>((n_sblk + wpb - 1) / wpb), L.n_chunks);
    hipLaunchKernelGGL((gen_kernel<DIST, DTYPE, ARITH, NT>), grid, dim3(L.block), 0, s, L);
    return hipGetLastError();
}

template <int DIST, int DTYPE>
static hipError_t launch_dd(const GenLaunch& L, hipStream_t s) {
    if (L.arith == kArithF64)
        return L.nontemporal ? launch_t<DIST, DTYPE, kArithF64, true>(L, s)
                             : launch_t<DIST, DTYPE, kArithF64, false>(L, s);
    return L.nontemporal ? launch_t<DIST, DTYPE, kArithInt, true>(L, s)
                         : launch_t<DIST, DTYPE, kArithInt, false>(L, s);
}

static hipError_t launch_gen_only(const GenLaunch& L, hipStream_t s) {
    switch (L.dist) {
        case kUniform:
            return L.dtype == kF64 ? launch_dd<kUniform, kF64>(L, s) : launch_dd<kUniform, kF32>(L, s);
        case kNormal:
            return L.dtype == kF64 ? launch_dd<kNormal, kF64>(L, s) : launch_dd<kNormal, kF32>(L, s);
        case kExponential:
            return L.dtype == kF64 ? launch_dd<kExponential, kF64>(L, s)
                                   : launch_dd<kExponential, kF32>(L, s);
        default:
            return launch_dd<kRaw, kU32>(L, s);
    }
}

hipError_t launch_generate(const GenLaunch& L, hipStream_t s) {
    if (L.n_chunks == 0) return hipSuccess;
    hipError_t e = launch_gen_only(L, s);
    if (e != hipSuccess || L.n_chunks == 1) return e;
    hipLaunchKernelGGL(finalize_kernel, dim3(grid1d(L.S, 256)), dim3(256), 0, s, L.streams, L.S, L.q,
                       L.r, L.dist == kNormal ? 1 : 0);
    return hipGetLastError();
}

}  // namespace mrg355
