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

#include <mutex>
#include <type_traits>

#include "mrg_engine.h"
#include "mrg_internal.h"
#include "mrg_math.h"
#include "mrg_tuned.h"

namespace mrg355 {

__constant__ JumpTables g_tab = make_jump_tables<kGen32k3a>();
__constant__ JumpTables g_tab31 = make_jump_tables<kGen31k3p>();
static constexpr JumpTables kHostTab = make_jump_tables<kGen32k3a>();
static constexpr JumpTables kHostTab31 = make_jump_tables<kGen31k3p>();
__constant__ StreamDigits g_dig = make_stream_digits<kGen32k3a>(kHostTab);
__constant__ StreamDigits g_dig31 = make_stream_digits<kGen31k3p>(kHostTab31);
__constant__ StepDigitsF64 g_stepdig = make_step_digits_f64<kGen32k3a>(kHostTab);
__constant__ StepDigitsF64 g_stepdig31 = make_step_digits_f64<kGen31k3p>(kHostTab31);

// ------------------------------------------------------------------ jumps
template <int G>
__device__ __forceinline__ const JumpTables& dev_tab() {
    if constexpr (G == kGen32k3a) return g_tab;
    else return g_tab31;
}

template <int G>
__device__ __forceinline__ const StreamDigits& dev_dig() {
    if constexpr (G == kGen32k3a) return g_dig;
    else return g_dig31;
}

// x <- (M1 x[0..2], M2 x[3..5]) modulo the generator's two moduli.
template <int G>
__device__ __forceinline__ void dev_apply(const Mat3& M1, const Mat3& M2, uint32_t x[6]) {
    if constexpr (G == kGen32k3a) {
        matvec<32>(M1, x, kC1);
        matvec<32>(M2, x + 3, kC2);
    } else {
        matvec<31>(M1, x, kQ1);
        matvec<31>(M2, x + 3, kQ2);
    }
}

// x <- A^e x, e wave-uniform.
template <int G>
__device__ __forceinline__ void dev_jump(uint32_t x[6], uint64_t e) {
    for (int b = 0; e; ++b, e >>= 1)
        if (e & 1) dev_apply<G>(dev_tab<G>().step_pow2[0][b], dev_tab<G>().step_pow2[1][b], x);
}

// x <- A^e x by base-64 digits of e: one exact fp64 matrix-vector product per
// nonzero digit instead of one integer product per set bit.  x canonical in
// and out.  Any e < 2^64 (the tables hold 11 digits); a wave-uniform e keeps
// the table reads scalar.
template <int G = kGen32k3a>
__device__ __forceinline__ void dev_jump_digits(uint32_t x[6], uint64_t e) {
    const StepDigitsF64& T = G == kGen32k3a ? g_stepdig : g_stepdig31;
    constexpr double m1 = G == kGen32k3a ? kM1d : static_cast<double>(kP1);
    constexpr double m2 = G == kGen32k3a ? kM2d : static_cast<double>(kP2);
    double v1[3] = {static_cast<double>(x[0]), static_cast<double>(x[1]), static_cast<double>(x[2])};
    double v2[3] = {static_cast<double>(x[3]), static_cast<double>(x[4]), static_cast<double>(x[5])};
    for (int d = 0; e; ++d, e >>= 6) {
        const uint32_t v = static_cast<uint32_t>(e & 63);
        if (v) {
            matvec_f64(T.m[d][0][v], v1, m1, 1.0 / m1);
            matvec_f64(T.m[d][1][v], v2, m2, 1.0 / m2);
        }
    }
#pragma unroll
    for (int w = 0; w < 3; ++w) {
        x[w] = static_cast<uint32_t>(v1[w]);
        x[3 + w] = static_cast<uint32_t>(v2[w]);
    }
}

// Largest float <= u (u in [2^-126, 1)) from v = u 2^-896, a normal double
// whose exponent field is already rebased from the double's bias to the
// float's (1023 - 127 = 896): the float is v's bits without the low 29
// mantissa bits.  Callers form v with the scale NORM 2^-896, which rounds
// exactly as NORM does (a power-of-two factor, no underflow for u >= 2^-126).
__device__ __forceinline__ float f32_rz_rebased(double v) {
    return __uint_as_float(static_cast<uint32_t>(static_cast<uint64_t>(__double_as_longlong(v)) >> 29));
}

template <int DTYPE> struct ElemOf;
template <> struct ElemOf<kF64> { using T = double; };
template <> struct ElemOf<kF32> { using T = float; };
template <> struct ElemOf<kU32> { using T = uint32_t; };

// The scale of Section 2.2 for generator G: 1/(m1+1).
template <int G>
__device__ __forceinline__ constexpr double norm_of() {
    return G == kGen32k3a ? kNorm : kNorm31;
}

// The stored value of one uniform / raw / exponential draw.
template <int DIST, int DTYPE, int G, typename Z>
__device__ __forceinline__ typename ElemOf<DTYPE>::T value1(Z z, double inv_rate) {
    if constexpr (DIST == kRaw) {
        return to_u32(z);
    } else if constexpr (DIST == kUniform && DTYPE == kF32) {
        return f32_rz_rebased(to_f64(z) * (norm_of<G>() * 0x1p-896));
    } else {
        double u = to_f64(z) * norm_of<G>();
        if constexpr (DIST == kExponential) {
            if constexpr (DTYPE == kF64) return -log_unit(u) * inv_rate;
            else return static_cast<float>(-log_unit_f32out(u) * inv_rate);
        } else {
            return u;
        }
    }
}

// Box-Muller pair (Algorithm 1) from two consecutive steps of one stream.
// The factors -2 and 2 are folded into exact power-of-two scalings: -2 log(u1)
// comes from log_unit<-2>, and 2 u2 = z2 (2 NORM) is the same double as
// 2 (z2 NORM).  A pair stored as floats (DTYPE kF32) takes the shorter
// evaluations of the same functions.
template <int G, int DTYPE, typename Z>
__device__ __forceinline__ void box_muller(Z z1, Z z2, double& x, double& y) {
    const double u1 = to_f64(z1) * norm_of<G>();
    const double t = to_f64(z2) * (2.0 * norm_of<G>());
    double r, s, c;
    if constexpr (DTYPE == kF64) {
        r = sqrt_radius(log_unit<-2>(u1));
        sincospi_unit(t, &s, &c);
    } else {
        r = sqrt_radius_f32out(log_unit_f32out<-2>(u1));
        sincospi_unit_f32out(t, &s, &c);
    }
    x = r * c;
    y = r * s;
}

template <int DTYPE>
__device__ __forceinline__ typename ElemOf<DTYPE>::T narrow(double v) {
    if constexpr (DTYPE == kF64) return v;
    else return static_cast<float>(v);
}

// ------------------------------------------------------------ row stores
// A row is the segment of one draw index that a wave writes: 64*SPL
// consecutive elements.  Stores go through a buffer resource whose base is
// the (wave-uniform, SGPR) row address and whose size is the rest of the row,
// so the per-lane offset is one fixed VGPR and no 64-bit address arithmetic
// runs per store.  An access past the row end would be dropped by hardware.
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <typename T, int N>
struct Pack {
    T v[N];
};

__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const char* row, uint32_t bytes) {
    // 0x00020000: 32-bit data format, as untyped buffer access expects on gfx9.
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<char*>(row), 0, static_cast<int>(bytes),
                                             0x00020000);
}

template <typename T, int N, bool NT>
__device__ __forceinline__ void store_n(__amdgpu_buffer_rsrc_t r, uint32_t voff, const Pack<T, N>& p) {
    constexpr int kAux = NT ? 2 : 0;  // nt bit
    constexpr int kBytes = N * static_cast<int>(sizeof(T));
    static_assert(kBytes == 4 || kBytes == 8 || kBytes == 16, "store width");
    if constexpr (kBytes == 4) {
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, p), r, voff, 0, kAux);
    } else if constexpr (kBytes == 8) {
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, p), r, voff, 0, kAux);
    } else {
        __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(u32x4, p), r, voff, 0, kAux);
    }
}

template <typename T, bool NT>
__device__ __forceinline__ void store_1(__amdgpu_buffer_rsrc_t r, uint32_t voff, T v) {
    Pack<T, 1> p{{v}};
    store_n<T, 1, NT>(r, voff, p);
}

// ------------------------------------------------------------ generate
// Draw units [u0, kend) of chunk `by` are the main-loop rows: every stream of
// the request has them (rows from kend on are the ragged tail).  Both bounds
// depend on the chunk only, so every wave of a block runs the same rows.
template <int DIST>
__device__ __forceinline__ void main_rows(const GenLaunch& L, uint32_t by, uint64_t& u0, uint64_t& u1,
                                          uint64_t& kend) {
    const uint64_t cnt_max = L.q + (L.r ? 1 : 0);
    const uint64_t units_max = DIST == kNormal ? (cnt_max + 1) / 2 : cnt_max;
    const uint64_t full = DIST == kNormal ? L.q / 2 : L.q;  // units every stream completes
    u0 = static_cast<uint64_t>(by) * L.chunk;
    u1 = min(u0 + L.chunk, units_max);
    kend = max(u0, min(u1, full));
}

// One wave = 64 lanes x SPL consecutive streams, one chunk of draw indices.
// Lane l owns streams s0 .. s0+SPL-1, s0 = first + l*SPL, and stores their
// SPL values of a draw index with one SPL*esz-byte store.
// One wave's share of one request: stream block `sblk` (64*SPL streams),
// draw units [by*chunk, (by+1)*chunk).  Wave-uniform arguments.
// LOCK: workgroup barriers per unrolled main-loop iteration (three rows, or
// three pairs for normals): 0, 1 (after the iteration) or 3 (after every row
// or pair).
template <int DIST, int DTYPE, int ARITH, int SPL, bool NT, int LOCK = 0>
__device__ __forceinline__ void run_chunk(const GenLaunch& L, uint32_t sblk, uint32_t by) {
    static_assert(LOCK == 0 || LOCK == 1 || LOCK == 3, "barriers per iteration");
    using Engine = typename std::conditional<
        ARITH == kArith31, Engine31,
        typename std::conditional<ARITH == kArithF64, F64Engine, IntEngine>::type>::type;
    constexpr int G = ARITH == kArith31 ? kGen31k3p : kGen32k3a;
    using T = typename ElemOf<DTYPE>::T;
    constexpr uint32_t ESZ = sizeof(T);
    constexpr uint32_t WS = 64 * SPL;                   // streams per wave
    constexpr uint64_t kSpu = DIST == kNormal ? 2 : 1;  // steps per unit
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t S = L.S;
    const uint32_t first = sblk * WS;
    const uint32_t s0 = first + lane * SPL;
    if (s0 >= S) return;  // S % SPL == 0: a lane's streams are all present or all absent

    // Work is counted in units: draws, or Box-Muller pairs for normals.
    uint64_t cnt[SPL], units[SPL];
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        cnt[i] = L.q + (s0 + i < L.r ? 1 : 0);
        units[i] = DIST == kNormal ? (cnt[i] + 1) / 2 : cnt[i];
    }
    uint64_t u0, u1, kend;
    main_rows<DIST>(L, by, u0, u1, kend);
    // Counts do not increase with s: stream s0 has the most.  A lane leaving
    // here has u0 >= q (>= q/2 for pairs), so kend == u0: no main-loop rows.
    if (u0 >= units[0]) return;

    Engine e[SPL];
#pragma unroll
    for (int i = 0; i < SPL; ++i) {
        const uint32_t* rec = L.streams + static_cast<uint64_t>(s0 + i) * 18;
        uint32_t x[6];
#pragma unroll
        for (int w = 0; w < 6; ++w) x[w] = rec[w];
        const uint64_t jump = L.offset + u0 * kSpu;
        if (jump) {
            // MRG31k3p keeps its per-bit jump here: with the digit tables
            // its main loop compiled about 5% slower at 262,144 x 4,096
            // (770 against 810 G uniforms/s), where no jump even runs
            if constexpr (ARITH == kArithF64) dev_jump_digits<G>(x, jump);
            else dev_jump<G>(x, jump);
        }
        e[i].load(x);
    }

    const double inv_rate = L.param;
    const uint64_t rowstep = static_cast<uint64_t>(S) * ESZ;
    const uint64_t rest = static_cast<uint64_t>(S - first) * ESZ;
    const uint32_t nrec = rest > 0xffffffffull ? 0xffffffffu : static_cast<uint32_t>(rest);
    const uint32_t voff = lane * SPL * ESZ;
    const char* row = static_cast<const char*>(L.out) + (u0 * kSpu * S + first) * ESZ;
    uint64_t k = u0;

    if constexpr (DIST == kNormal) {
        // 3 pairs = 6 steps per iteration: the register ring returns home.
        // Each pair is transformed and stored as soon as its two steps exist,
        // which keeps few values live.
        auto pair = [&](auto z_of) {
            Pack<T, SPL> px, py;
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                double x, y;
                z_of(e[i], x, y);
                px.v[i] = narrow<DTYPE>(x);
                py.v[i] = narrow<DTYPE>(y);
            }
            store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, px);
            row += rowstep;
            store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, py);
            row += rowstep;
            if constexpr (LOCK == 3) __builtin_amdgcn_s_barrier();
        };
        for (; k + 3 <= kend; k += 3) {
            pair([](Engine& g, double& x, double& y) {
                auto z0 = g.template step<0>();
                auto z1 = g.template step<1>();
                box_muller<G, DTYPE>(z0, z1, x, y);
            });
            pair([](Engine& g, double& x, double& y) {
                auto z2 = g.template step<2>();
                auto z3 = g.template step<0>();
                box_muller<G, DTYPE>(z2, z3, x, y);
            });
            pair([](Engine& g, double& x, double& y) {
                auto z4 = g.template step<1>();
                auto z5 = g.template step<2>();
                box_muller<G, DTYPE>(z4, z5, x, y);
            });
            if constexpr (LOCK == 1) __builtin_amdgcn_s_barrier();
        }
        for (; k < kend; ++k) {
            Pack<T, SPL> px, py;
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                auto z0 = e[i].step_rot();
                auto z1 = e[i].step_rot();
                double x, y;
                box_muller<G, DTYPE>(z0, z1, x, y);
                px.v[i] = narrow<DTYPE>(x);
                py.v[i] = narrow<DTYPE>(y);
            }
            store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, px);
            row += rowstep;
            store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, py);
            row += rowstep;
        }
        // Ragged tail (at most one pair): X and Y only where they exist.
        const uint64_t tend = min(u1, units[0]);
        for (; k < tend; ++k) {
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                if (k < units[i]) {
                    auto z0 = e[i].step_rot();
                    auto z1 = e[i].step_rot();
                    double x, y;
                    box_muller<G, DTYPE>(z0, z1, x, y);
                    if (2 * k < cnt[i]) store_1<T, NT>(row_rsrc(row, nrec), voff + i * ESZ, narrow<DTYPE>(x));
                    if (2 * k + 1 < cnt[i])
                        store_1<T, NT>(row_rsrc(row + rowstep, nrec), voff + i * ESZ, narrow<DTYPE>(y));
                }
            }
            row += 2 * rowstep;
        }
    } else {
        for (; k + 3 <= kend; k += 3) {
            Pack<T, SPL> p0, p1, p2;
#pragma unroll
            for (int i = 0; i < SPL; ++i) {
                p0.v[i] = value1<DIST, DTYPE, G>(e[i].template step<0>(), inv_rate);
                p1.v[i] = value1<DIST, DTYPE, G>(e[i].template step<1>(), inv_rate);
                p2.v[i] = value1<DIST, DTYPE, G>(e[i].template step<2>(), inv_rate);
            }
            store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, p0);
            row += rowstep;
            if constexpr (LOCK == 3) __builtin_amdgcn_s_barrier();
            store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, p1);
            row += rowstep;
            if constexpr (LOCK == 3) __builtin_amdgcn_s_barrier();
            store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, p2);
            row += rowstep;
            if constexpr (LOCK != 0) __builtin_amdgcn_s_barrier();
        }
        for (; k < kend; ++k) {
            Pack<T, SPL> p;
#pragma unroll
            for (int i = 0; i < SPL; ++i) p.v[i] = value1<DIST, DTYPE, G>(e[i].step_rot(), inv_rate);
            store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, p);
            row += rowstep;
        }
        const uint64_t tend = min(u1, units[0]);
        for (; k < tend; ++k) {
#pragma unroll
            for (int i = 0; i < SPL; ++i)
                if (k < units[i])
                    store_1<T, NT>(row_rsrc(row, nrec), voff + i * ESZ,
                                   value1<DIST, DTYPE, G>(e[i].step_rot(), inv_rate));
            row += rowstep;
        }
    }

    // A stream owned by a single work-item is written back here; otherwise
    // finalize_kernel advances it after this launch (other chunks of the same
    // stream may not have read it yet).
    if (L.n_chunks == 1 && !L.no_writeback) {
#pragma unroll
        for (int i = 0; i < SPL; ++i) {
            uint32_t x[6];
            e[i].save(x);
            uint32_t* rec = L.streams + static_cast<uint64_t>(s0 + i) * 18;
#pragma unroll
            for (int w = 0; w < 6; ++w) rec[w] = x[w];
        }
    }
}

// LOCK: the waves of a block pass a barrier after each row of the main
// loops (three per unrolled iteration), so a block writes 64*SPL*waves
// consecutive elements of a row at once.  All waves of a block run the same
// main-loop rows (main_rows); a wave past the last stream block stays to
// pass the same barriers, and lanes past the last stream leave without
// ending their wave (a wave's lane 0 always holds a stream).
template <int DIST, int DTYPE, int ARITH, int SPL, bool NT, bool LOCK>
__global__ void __launch_bounds__(1024) gen_kernel(GenLaunch L) {
    if constexpr (DIST == kNormal || DIST == kExponential) stage_tables();
    // Block -> (stream block, chunk).  With xcd remapping, consecutive logical
    // blocks (neighbouring row segments) land on one XCD, whose L2 then sees
    // contiguous runs of every row; blocks are dealt to the 8 XCDs in turn.
    uint32_t bx = blockIdx.x, by = blockIdx.y;
    if (L.xcd) {
        const uint32_t total = gridDim.x * gridDim.y;
        uint32_t lin = blockIdx.x + blockIdx.y * gridDim.x;
        lin = (lin % 8) * (total / 8) + lin / 8;  // host guarantees total % 8 == 0
        bx = lin % gridDim.x;
        by = lin / gridDim.x;
    }
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t sblk = bx * (blockDim.x >> 6) + wave;
    if (sblk >= (L.S + 64 * SPL - 1) / (64 * SPL)) {
        if constexpr (LOCK) {
            uint64_t u0, u1, kend;
            main_rows<DIST>(L, by, u0, u1, kend);
            for (uint64_t k = u0; k + 3 <= kend; k += 3) {
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_s_barrier();
                __builtin_amdgcn_s_barrier();
            }
        }
        return;
    }
    run_chunk<DIST, DTYPE, ARITH, SPL, NT, LOCK ? 3 : 0>(L, sblk, by);
}

// cur <- A^(steps consumed) cur for every stream, after a chunked launch:
// cnt_s = q + (s < r) draws; normals consume 2*ceil(cnt_s/2) steps.
template <int G>
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
    dev_jump_digits<G>(x, steps);  // lanes hold one or two distinct counts
#pragma unroll
    for (int w = 0; w < 6; ++w) rec[w] = x[w];
}

// --------------------------------------------------------------- batching
// Counters of every request are reset at the start of each launch by a small
// kernel (no memset node, so the launch can be captured in a graph).
__global__ void __launch_bounds__(256) batch_init_kernel(BatchLaunch B) {
    uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && B.n_gangs) {
        // gang mode: block b, the (b / 8)-th block on XCD b mod 8, starts on
        // that XCD's gang b / 8; each XCD's queue hands out the rest
        for (int x = 0; x < kXcdQueues; ++x) {
            const uint32_t blocks = B.grid > static_cast<uint32_t>(x) ? (B.grid - x + kXcdQueues - 1) / kXcdQueues : 0;
            const uint32_t count = B.xq_lo[x + 1] - B.xq_lo[x];
            B.head->queue[x] = blocks < count ? blocks : count;
        }
        B.head->t_start = 0;
    } else if (i == 0) {
        // tiles [0, waves of the class) are taken without the queue (each
        // wave's first tile in its own class); the queue hands out the rest
        for (int c = 0; c < kClasses; ++c) {
            const uint32_t waves = (B.block_lo[c + 1] - B.block_lo[c]) * B.wpb;
            const uint32_t count = B.tile_lo[c + 1] - B.tile_lo[c];
            B.head->queue[c] = waves < count ? waves : count;
        }
        for (int c = kClasses; c < kXcdQueues; ++c) B.head->queue[c] = 0;
        B.head->t_start = 0;
    }
    if (i < B.n_req) {
        B.slots[i].remaining = B.reqs[i].n_tiles;
        B.slots[i].done = 0;
        B.slots[i].t_done = 0;
    }
}

// Batch tiles use ordinary stores: requests of a few hundred streams have rows
// that seldom start on a 128-byte line, and L2 then merges the halves of the
// line two neighbouring tiles share (4,096-request mix: 9.97 ms against 10.30 ms with
// non-temporal stores; f32 uniforms 1.34 against 1.71 ms).
template <int KIND>
__device__ __forceinline__ void batch_tile(const GenLaunch& L, uint32_t sblk, uint32_t chunk) {
    if constexpr (KIND == kBUniF64x1) run_chunk<kUniform, kF64, kArithF64, 1, false>(L, sblk, chunk);
    if constexpr (KIND == kBUniF64x2) run_chunk<kUniform, kF64, kArithF64, 2, false>(L, sblk, chunk);
    if constexpr (KIND == kBUniF32x1) run_chunk<kUniform, kF32, kArithF64, 1, false>(L, sblk, chunk);
    if constexpr (KIND == kBUniF32x4) run_chunk<kUniform, kF32, kArithF64, 4, false>(L, sblk, chunk);
    if constexpr (KIND == kBRawU32x1) run_chunk<kRaw, kU32, kArithF64, 1, false>(L, sblk, chunk);
    if constexpr (KIND == kBRawU32x4) run_chunk<kRaw, kU32, kArithF64, 4, false>(L, sblk, chunk);
    if constexpr (KIND == kBNormF64) run_chunk<kNormal, kF64, kArithF64, 1, false>(L, sblk, chunk);
    if constexpr (KIND == kBNormF32) run_chunk<kNormal, kF32, kArithF64, 1, false>(L, sblk, chunk);
    if constexpr (KIND == kBExpF64) run_chunk<kExponential, kF64, kArithF64, 1, false>(L, sblk, chunk);
    if constexpr (KIND == kBExpF32) run_chunk<kExponential, kF32, kArithF64, 1, false>(L, sblk, chunk);
    if constexpr (KIND == kBNormF64x2) run_chunk<kNormal, kF64, kArithF64, 2, false>(L, sblk, chunk);
    if constexpr (KIND == kBNormF32x2) run_chunk<kNormal, kF32, kArithF64, 2, false>(L, sblk, chunk);
    if constexpr (KIND == kBExpF64x2) run_chunk<kExponential, kF64, kArithF64, 2, false>(L, sblk, chunk);
    if constexpr (KIND == kBExpF32x2) run_chunk<kExponential, kF32, kArithF64, 2, false>(L, sblk, chunk);
}

// A wave has stored its tile of request `req`: count the tile off the request;
// the wave that finishes the request stamps the device real-time clock into its
// slot.  `one` is 1 on lane 0 and 0 elsewhere (every lane executes the atomic).
__device__ __forceinline__ void finish_tile(const BatchLaunch& B, uint32_t req, uint32_t one) {
    // The count must follow this wave's stores.  When a host thread watches
    // completions (serving), it may hand a finished output to other work while
    // this kernel still runs: the stores are released device-wide (an L2
    // write-back on this chip).  Otherwise consumers are ordered after the
    // launch, whose end makes everything visible, and waiting for the stores
    // to complete is enough.
    if (B.host_slots) __threadfence();
    else __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    const uint32_t left = __builtin_amdgcn_readfirstlane(atomicSub(&B.slots[req].remaining, one));
    if (left == 1) {  // wave-uniform: this wave finished the request
        const uint64_t t_done = __builtin_amdgcn_s_memrealtime();
        B.slots[req].t_done = t_done;
        __threadfence();
        B.slots[req].done = 1;
        if (B.host_slots) {  // tell a polling host thread
            B.host_slots[req].t_done = t_done;
            __threadfence_system();
            B.host_slots[req].done = 1;
        }
    }
}

// Persistent kernel.  Tiles come in three classes with separate queues:
// normals, exponentials (both fp64-transcendental heavy) and uniform/raw.
// Each class has its own loop, which contains only that class's code, so the
// register budget of the kernel is that of its largest class rather than of
// all of them together (constants hoisted above a loop stay live for the
// whole loop).  Within a class, every wave takes
// tiles from one atomic counter until the class queue is empty (at most
// (tiles of the class) + 1 takes per wave).  Tiles were sorted longest first
// on the host.  After its stores, a wave counts the tile off its request; the
// wave that finishes a request stamps the device real-time clock into the
// request's slot.
//
// No branch on the lane index surrounds the atomics: every lane executes them
// with an increment of 1 on lane 0 and 0 elsewhere, and the wave takes lane
// 0's result with readfirstlane.  Each loop's control flow is therefore
// wave-uniform, and no lane can be left iterating on its own.
template <int CLS>
__device__ __forceinline__ void batch_worker(const BatchLaunch& B, uint32_t first) {
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t one = lane == 0 ? 1u : 0u;
    const uint32_t lo = B.tile_lo[CLS];
    const uint32_t count = B.tile_lo[CLS + 1] - lo;
    uint32_t* queue = &B.head->queue[CLS];
    for (;;) {
        // the first tile of a wave in its own class is its rank there (no
        // atomic); every other tile comes from the queue
        const uint32_t q = first != 0xffffffffu ? first : __builtin_amdgcn_readfirstlane(atomicAdd(queue, one));
        first = 0xffffffffu;
        if (q >= count) break;
        const uint32_t t = lo + q;
        const uint32_t req = __builtin_amdgcn_readfirstlane(B.tiles[t].req);
        const uint32_t sblk = __builtin_amdgcn_readfirstlane(B.tiles[t].sblk);
        const uint32_t chunk = __builtin_amdgcn_readfirstlane(B.tiles[t].chunk);
        const uint32_t kind = __builtin_amdgcn_readfirstlane(B.reqs[req].kind);
        const GenLaunch& L = B.reqs[req].L;
        if constexpr (CLS == kClsNormal) {
            switch (kind) {
                case kBNormF64: batch_tile<kBNormF64>(L, sblk, chunk); break;
                case kBNormF32: batch_tile<kBNormF32>(L, sblk, chunk); break;
                case kBNormF64x2: batch_tile<kBNormF64x2>(L, sblk, chunk); break;
                default: batch_tile<kBNormF32x2>(L, sblk, chunk); break;
            }
        } else if constexpr (CLS == kClsExp) {
            switch (kind) {
                case kBExpF64: batch_tile<kBExpF64>(L, sblk, chunk); break;
                case kBExpF32: batch_tile<kBExpF32>(L, sblk, chunk); break;
                case kBExpF64x2: batch_tile<kBExpF64x2>(L, sblk, chunk); break;
                default: batch_tile<kBExpF32x2>(L, sblk, chunk); break;
            }
        } else {
            switch (kind) {
                case kBUniF64x1: batch_tile<kBUniF64x1>(L, sblk, chunk); break;
                case kBUniF64x2: batch_tile<kBUniF64x2>(L, sblk, chunk); break;
                case kBUniF32x1: batch_tile<kBUniF32x1>(L, sblk, chunk); break;
                case kBUniF32x4: batch_tile<kBUniF32x4>(L, sblk, chunk); break;
                case kBRawU32x1: batch_tile<kBRawU32x1>(L, sblk, chunk); break;
                default: batch_tile<kBRawU32x4>(L, sblk, chunk); break;
            }
        }
        finish_tile(B, req, one);
    }
}

// A wave's rank among the waves of its own class, blocks ordered so that each
// XCD (physical block b runs on XCD b mod 8) takes a contiguous run of the
// class's tiles when the class's blocks allow it.
__device__ __forceinline__ uint32_t home_rank(const BatchLaunch& B, int cls) {
    const uint32_t b0 = B.block_lo[cls], nb = B.block_lo[cls + 1] - b0;
    uint32_t i = blockIdx.x - b0;
    if (b0 % 8 == 0 && nb % 8 == 0) i = (i % 8) * (nb / 8) + i / 8;
    return i * B.wpb + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
}

// A block starts on its own class (blocks are shared out by estimated work),
// then helps the other classes until every queue is empty.  The three loops
// run one after another, so their register live ranges never overlap.
__global__ void __launch_bounds__(256) batch_kernel(BatchLaunch B) {
    stage_tables();
    constexpr uint32_t kNone = 0xffffffffu;
    if (blockIdx.x == 0 && threadIdx.x < 64) B.head->t_start = __builtin_amdgcn_s_memrealtime();
    if (blockIdx.x < B.block_lo[1]) {
        batch_worker<kClsNormal>(B, home_rank(B, kClsNormal));
        batch_worker<kClsExp>(B, kNone);
        batch_worker<kClsPlain>(B, kNone);
    } else if (blockIdx.x < B.block_lo[2]) {
        batch_worker<kClsExp>(B, home_rank(B, kClsExp));
        batch_worker<kClsNormal>(B, kNone);
        batch_worker<kClsPlain>(B, kNone);
    } else {
        batch_worker<kClsPlain>(B, home_rank(B, kClsPlain));
        batch_worker<kClsNormal>(B, kNone);
        batch_worker<kClsExp>(B, kNone);
    }
}

// ---------------------------------------------------------- gang batching
// A gang is G wave tiles (G = waves per block) that one block runs together:
// wave w takes tile w of the gang, and the waves pass a workgroup barrier after
// every three rows (pairs, for normals) of their main loops.  The host puts consecutive
// stream blocks of one request and chunk in a gang, so the row segments of
// neighbouring waves -- which share a cache line wherever a row does not start
// on a 128-byte line -- are written within a few rows of each other and the
// line is completed in this CU's L2 instead of reaching HBM in two partial
// writes.  Every wave passes as many barriers as the gang's longest main loop
// (each wave works out every tile's count with the rule run_chunk follows).
// Gangs of every class share one queue, which the host interleaves so that the
// classes advance at the same pace: transform-heavy and store-heavy tiles run
// side by side throughout the launch and finish together.
// One barrier per unrolled iteration (three rows) rather than per row: the
// 4,096-request mix ran 7.49 ms against 7.53 ms (gangs of 8, one stream per
// lane); with none at all, waves drift apart and the shared lines are no
// longer completed in L2.
#ifndef MRG_GANG_LOCK
#define MRG_GANG_LOCK 1
#endif
constexpr int kGangLock = MRG_GANG_LOCK;  // barriers per unrolled main-loop iteration (0, 1 or 3)

template <int KIND>
__device__ __forceinline__ void gang_tile(const GenLaunch& L, uint32_t sblk, uint32_t chunk) {
    if constexpr (KIND == kBUniF64x1) run_chunk<kUniform, kF64, kArithF64, 1, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBUniF64x2) run_chunk<kUniform, kF64, kArithF64, 2, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBUniF32x1) run_chunk<kUniform, kF32, kArithF64, 1, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBUniF32x4) run_chunk<kUniform, kF32, kArithF64, 4, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBRawU32x1) run_chunk<kRaw, kU32, kArithF64, 1, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBRawU32x4) run_chunk<kRaw, kU32, kArithF64, 4, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBNormF64) run_chunk<kNormal, kF64, kArithF64, 1, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBNormF32) run_chunk<kNormal, kF32, kArithF64, 1, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBExpF64) run_chunk<kExponential, kF64, kArithF64, 1, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBExpF32) run_chunk<kExponential, kF32, kArithF64, 1, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBNormF64x2) run_chunk<kNormal, kF64, kArithF64, 2, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBNormF32x2) run_chunk<kNormal, kF32, kArithF64, 2, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBExpF64x2) run_chunk<kExponential, kF64, kArithF64, 2, false, kGangLock>(L, sblk, chunk);
    if constexpr (KIND == kBExpF32x2) run_chunk<kExponential, kF32, kArithF64, 2, false, kGangLock>(L, sblk, chunk);
}

// Main-loop iterations of a wave tile: run_chunk passes kGangLock barriers
// per iteration, and its main loop runs floor((kend - u0) / 3) of them, with u0
// and kend as main_rows gives them (0 for the padding of a short gang).  Every
// operand is wave-uniform.
__device__ __forceinline__ uint32_t tile_iters(const BatchLaunch& B, const BatchTile& T) {
    const uint32_t req = __builtin_amdgcn_readfirstlane(T.req);
    if (req == kNoRequest) return 0;
    const GenLaunch& L = B.reqs[req].L;
    const uint32_t chunk = __builtin_amdgcn_readfirstlane(T.chunk);
    uint64_t u0, u1, kend;
    if (L.dist == kNormal) main_rows<kNormal>(L, chunk, u0, u1, kend);
    else main_rows<kUniform>(L, chunk, u0, u1, kend);
    return __builtin_amdgcn_readfirstlane(static_cast<uint32_t>((kend - u0) / 3));
}

// Gangs come from one queue per XCD: the host gives each request's gangs to
// one XCD, so that the lines two of its gangs share are completed in that
// XCD's L2, and a block takes its own XCD's gangs first (block b runs on XCD
// b mod 8, the (b / 8)-th there, and starts on that list's gang b / 8), then
// those of the others in turn until every list is empty.  The gang index
// travels through LDS: wave 0 takes it (every lane executes the atomics,
// increment 1 on lane 0 only), and two barriers bracket the read so that no
// wave can overwrite it before every wave has read it.  All control flow
// around the barriers is block-uniform.
//
// NARROW: the plan holds only tiles of one stream per lane.  Their code alone
// fits the registers of six resident waves per SIMD, where the code of every
// kind together allows three.
template <bool NARROW>
__device__ __forceinline__ void gang_loop(const BatchLaunch& B) {
    stage_tables();
    __shared__ uint32_t next_gang;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t one = lane == 0 ? 1u : 0u;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    if (blockIdx.x == 0 && threadIdx.x < 64) B.head->t_start = __builtin_amdgcn_s_memrealtime();
    constexpr uint32_t kFetch = 0xfffffffeu, kNone = 0xffffffffu;
    const uint32_t home = blockIdx.x % kXcdQueues;
    const uint32_t rank = blockIdx.x / kXcdQueues;
    uint32_t g = rank < B.xq_lo[home + 1] - B.xq_lo[home] ? B.xq_lo[home] + rank : kFetch;
    for (;;) {
        if (g == kFetch) {
            if (wave == 0) {
                uint32_t nxt = kNone;
                for (uint32_t y = 0; y < kXcdQueues && nxt == kNone; ++y) {
                    const uint32_t x = (home + y) % kXcdQueues;
                    const uint32_t count = B.xq_lo[x + 1] - B.xq_lo[x];
                    const uint32_t q = __builtin_amdgcn_readfirstlane(atomicAdd(&B.head->queue[x], one));
                    if (q < count) nxt = B.xq_lo[x] + q;
                }
                next_gang = nxt;
            }
            __syncthreads();
            g = next_gang;
            __syncthreads();
        }
        if (g == kNone) break;
        const BatchTile* gt = B.tiles + static_cast<uint64_t>(g) * B.wpb;
        uint32_t nbar = 0, nit = 0;
        for (uint32_t w = 0; w < B.wpb; ++w) {
            const uint32_t it = tile_iters(B, gt[w]);
            nbar = it > nbar ? it : nbar;
            if (w == wave) nit = it;
        }
        const uint32_t req = __builtin_amdgcn_readfirstlane(gt[wave].req);
        if (req != kNoRequest) {
            const uint32_t sblk = __builtin_amdgcn_readfirstlane(gt[wave].sblk);
            const uint32_t chunk = __builtin_amdgcn_readfirstlane(gt[wave].chunk);
            const uint32_t kind = __builtin_amdgcn_readfirstlane(B.reqs[req].kind);
            const GenLaunch& L = B.reqs[req].L;
            if constexpr (NARROW) {
                switch (kind) {
                    case kBUniF64x1: gang_tile<kBUniF64x1>(L, sblk, chunk); break;
                    case kBUniF32x1: gang_tile<kBUniF32x1>(L, sblk, chunk); break;
                    case kBRawU32x1: gang_tile<kBRawU32x1>(L, sblk, chunk); break;
                    case kBNormF64: gang_tile<kBNormF64>(L, sblk, chunk); break;
                    case kBNormF32: gang_tile<kBNormF32>(L, sblk, chunk); break;
                    case kBExpF64: gang_tile<kBExpF64>(L, sblk, chunk); break;
                    default: gang_tile<kBExpF32>(L, sblk, chunk); break;
                }
            } else {
                switch (kind) {
                    case kBUniF64x1: gang_tile<kBUniF64x1>(L, sblk, chunk); break;
                    case kBUniF64x2: gang_tile<kBUniF64x2>(L, sblk, chunk); break;
                    case kBUniF32x1: gang_tile<kBUniF32x1>(L, sblk, chunk); break;
                    case kBUniF32x4: gang_tile<kBUniF32x4>(L, sblk, chunk); break;
                    case kBRawU32x1: gang_tile<kBRawU32x1>(L, sblk, chunk); break;
                    case kBRawU32x4: gang_tile<kBRawU32x4>(L, sblk, chunk); break;
                    case kBNormF64: gang_tile<kBNormF64>(L, sblk, chunk); break;
                    case kBNormF32: gang_tile<kBNormF32>(L, sblk, chunk); break;
                    case kBExpF64: gang_tile<kBExpF64>(L, sblk, chunk); break;
                    case kBExpF32: gang_tile<kBExpF32>(L, sblk, chunk); break;
                    case kBNormF64x2: gang_tile<kBNormF64x2>(L, sblk, chunk); break;
                    case kBNormF32x2: gang_tile<kBNormF32x2>(L, sblk, chunk); break;
                    case kBExpF64x2: gang_tile<kBExpF64x2>(L, sblk, chunk); break;
                    default: gang_tile<kBExpF32x2>(L, sblk, chunk); break;
                }
            }
            finish_tile(B, req, one);
        }
        // the barriers of the gang's longer main loops (kGangLock per
        // unrolled iteration, as run_chunk passes them)
        if constexpr (kGangLock != 0) {
            for (uint32_t i = nit; i < nbar; ++i) {
                __builtin_amdgcn_s_barrier();
                if constexpr (kGangLock == 3) {
                    __builtin_amdgcn_s_barrier();
                    __builtin_amdgcn_s_barrier();
                }
            }
        }
        g = kFetch;
    }
}

__global__ void __launch_bounds__(512) batch_gang_kernel(BatchLaunch B) { gang_loop<false>(B); }

__global__ void __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(6)))
batch_gang_narrow_kernel(BatchLaunch B) {
    gang_loop<true>(B);
}

// States of requests split over several chunks: cur <- A^(steps consumed) cur,
// after every tile has read them.  Thread g -> (request, stream) through the
// prefix sums of their stream counts.
__global__ void __launch_bounds__(256) batch_finalize_kernel(BatchLaunch B) {
    const uint64_t g = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g >= B.fin_total) return;
    uint32_t lo = 0, hi = B.n_fin;  // largest i with fin_pre[i] <= g
    while (hi - lo > 1) {
        uint32_t mid = (lo + hi) / 2;
        if (B.fin_pre[mid] <= g) lo = mid;
        else hi = mid;
    }
    const GenLaunch& L = B.reqs[B.fin_req[lo]].L;
    const uint32_t s = static_cast<uint32_t>(g - B.fin_pre[lo]);
    const uint64_t cnt = L.q + (s < L.r ? 1 : 0);
    const uint64_t steps = L.dist == kNormal ? (cnt + 1) / 2 * 2 : cnt;
    uint32_t* rec = L.streams + static_cast<uint64_t>(s) * 18;
    uint32_t x[6];
#pragma unroll
    for (int w = 0; w < 6; ++w) x[w] = rec[w];
    dev_jump_digits<kGen32k3a>(x, steps);
#pragma unroll
    for (int w = 0; w < 6; ++w) rec[w] = x[w];
}

// ------------------------------------------------------ stream creation
// Stream i = J^i creator with J = A^Z (Z = 2^127, or 2^134 for MRG31k3p),
// in two steps: stream 64w (the first stream of each group of 64), then
// stream 64w + l = J^l times it.  J^i is the product of one table entry per
// nonzero base-64 digit of i (StreamDigits: J^(v 64^d)): at most five
// matrix-vector products for a group's first stream (i < 2^36), one per lane.
template <int G>
__device__ __forceinline__ void write_record(uint32_t* rec, const uint32_t x[6]) {
#pragma unroll
    for (int w = 0; w < 6; ++w) {
        rec[w] = x[w];
        rec[6 + w] = x[w];
        rec[12 + w] = x[w];
    }
}

// Copy digit tables [first, first + count) of both components into LDS as
// doubles (each lane picks its own entry, so they cannot be scalar loads);
// creation then multiplies in fp64 (matvec_f64: the same integers as the
// 64-bit integer products, with a third of the instructions).
template <int G>
__device__ __forceinline__ void stage_digit_tables(double (*dst)[64][2][9], int first, int count) {
    for (int k = threadIdx.x; k < count * 64 * 9; k += blockDim.x) {
        const int d = k / (64 * 9), v = (k / 9) % 64, e = k % 9;
        dst[d][v][0][e] = static_cast<double>(dev_dig<G>().digit[first + d][0][v].a[e]);
        dst[d][v][1][e] = static_cast<double>(dev_dig<G>().digit[first + d][1][v].a[e]);
    }
    __syncthreads();
}

template <int G>
__device__ __forceinline__ void apply_f64(const double (&M)[2][9], double x[6]) {
    constexpr double m1 = G == kGen32k3a ? static_cast<double>(kM1) : static_cast<double>(kP1);
    constexpr double m2 = G == kGen32k3a ? static_cast<double>(kM2) : static_cast<double>(kP2);
    matvec_f64(M[0], x, m1, 1.0 / m1);
    matvec_f64(M[1], x + 3, m2, 1.0 / m2);
}

// Both passes in one launch: a block's 256 streams are four groups of 64,
// whose first streams it makes itself (lanes 0-3, one product per nonzero
// digit of the group index, the tables read from global memory), so no block
// reads another's records.
template <int G>
__global__ void __launch_bounds__(256) create_kernel(uint32_t* out, uint64_t n, uint32_t c0, uint32_t c1,
                                                     uint32_t c2, uint32_t c3, uint32_t c4, uint32_t c5,
                                                     int ndig) {
    __shared__ double tab[1][64][2][9];  // J^v, v < 64
    __shared__ double gstart[4][6];      // streams 64 g of the block's groups
    __shared__ uint32_t recs[256 * 18];
    const uint64_t first_i = static_cast<uint64_t>(blockIdx.x) * 256;
    if (threadIdx.x < 4) {
        const uint64_t g = first_i / 64 + threadIdx.x;
        double x[6] = {static_cast<double>(c0), static_cast<double>(c1), static_cast<double>(c2),
                       static_cast<double>(c3), static_cast<double>(c4), static_cast<double>(c5)};
        if (g * 64 < n) {
            for (int d = 0; d < ndig; ++d) {  // digit d of g is digit d + 1 of the stream index
                const uint32_t v = static_cast<uint32_t>(g >> (6 * d)) & 63u;
                if (v) {
                    double M[2][9];
#pragma unroll
                    for (int e = 0; e < 9; ++e) {
                        M[0][e] = static_cast<double>(dev_dig<G>().digit[d + 1][0][v].a[e]);
                        M[1][e] = static_cast<double>(dev_dig<G>().digit[d + 1][1][v].a[e]);
                    }
                    apply_f64<G>(M, x);
                }
            }
        }
#pragma unroll
        for (int w = 0; w < 6; ++w) gstart[threadIdx.x][w] = x[w];
    }
    stage_digit_tables<G>(tab, 0, 1);  // ends with a barrier every thread reaches: gstart is written
    const uint64_t i = first_i + threadIdx.x;
    if (i < n) {
        double x[6];
#pragma unroll
        for (int w = 0; w < 6; ++w) x[w] = gstart[threadIdx.x >> 6][w];
        const uint32_t v = static_cast<uint32_t>(i) & 63u;
        if (v) apply_f64<G>(tab[0][v], x);
        uint32_t w[6];
#pragma unroll
        for (int k = 0; k < 6; ++k) w[k] = static_cast<uint32_t>(x[k]);
        write_record<G>(recs + threadIdx.x * 18, w);
    }
    __syncthreads();
    const uint64_t n_here = n - first_i < 256 ? n - first_i : 256;
    const uint32_t words = static_cast<uint32_t>(n_here) * 18;
    uint32_t* dst = out + first_i * 18;
    for (uint32_t k = threadIdx.x; k < words; k += 256) dst[k] = recs[k];
}

template <int G>
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
        if (kind == 2) dev_apply<G>(dev_tab<G>().substream[0], dev_tab<G>().substream[1], x);
    }
#pragma unroll
    for (int w = 0; w < 6; ++w) {
        rec[w] = x[w];
        rec[12 + w] = x[w];
    }
}

template <int G>
__global__ void __launch_bounds__(256) advance_kernel(uint32_t* streams, uint64_t n, uint64_t steps) {
    uint64_t i = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t* rec = streams + i * 18;
    uint32_t x[6];
#pragma unroll
    for (int w = 0; w < 6; ++w) x[w] = rec[w];
    dev_jump_digits<G>(x, steps);
#pragma unroll
    for (int w = 0; w < 6; ++w) rec[w] = x[w];
}

// ------------------------------------------------------------ host side
void host_jump_pow2(int gen, uint32_t state[6], uint64_t k, bool stream_tables) {
    const JumpTables& T = gen == kGen32k3a ? kHostTab : kHostTab31;
    for (int b = 0; k; ++b, k >>= 1) {
        if (!(k & 1)) continue;
        const Mat3& A = stream_tables ? T.stream_pow2[0][b] : T.step_pow2[0][b];
        const Mat3& B = stream_tables ? T.stream_pow2[1][b] : T.step_pow2[1][b];
        if (gen == kGen32k3a) {
            matvec<32>(A, state, kC1);
            matvec<32>(B, state + 3, kC2);
        } else {
            matvec<31>(A, state, kQ1);
            matvec<31>(B, state + 3, kQ2);
        }
    }
}

static unsigned grid1d(uint64_t n, unsigned block) {
    return static_cast<unsigned>((n + block - 1) / block);
}

template <int G>
static hipError_t launch_create_t(uint32_t* out, uint64_t n, const uint32_t c[6], hipStream_t s) {
    const uint64_t groups = (n + 63) / 64;
    int ndig = 0;  // base-64 digits of the largest group index
    while (ndig < kStreamDigits && ((groups - 1) >> (6 * ndig))) ++ndig;
    if (ndig > kStreamDigits - 1) return hipErrorInvalidValue;  // more than 2^36 streams (refused by the API)
    hipLaunchKernelGGL(create_kernel<G>, dim3(grid1d(n, 256)), dim3(256), 0, s, out, n, c[0], c[1], c[2], c[3],
                       c[4], c[5], ndig);
    return hipGetLastError();
}

hipError_t launch_create(int gen, uint32_t* out, uint64_t n, const uint32_t c[6], hipStream_t s) {
    return gen == kGen32k3a ? launch_create_t<kGen32k3a>(out, n, c, s) : launch_create_t<kGen31k3p>(out, n, c, s);
}

hipError_t launch_reset(int gen, uint32_t* streams, uint64_t n, int kind, hipStream_t s) {
    if (gen == kGen32k3a)
        hipLaunchKernelGGL(reset_kernel<kGen32k3a>, dim3(grid1d(n, 256)), dim3(256), 0, s, streams, n, kind);
    else
        hipLaunchKernelGGL(reset_kernel<kGen31k3p>, dim3(grid1d(n, 256)), dim3(256), 0, s, streams, n, kind);
    return hipGetLastError();
}

hipError_t launch_advance(int gen, uint32_t* streams, uint64_t n, uint64_t steps, hipStream_t s) {
    if (gen == kGen32k3a)
        hipLaunchKernelGGL(advance_kernel<kGen32k3a>, dim3(grid1d(n, 256)), dim3(256), 0, s, streams, n, steps);
    else
        hipLaunchKernelGGL(advance_kernel<kGen31k3p>, dim3(grid1d(n, 256)), dim3(256), 0, s, streams, n, steps);
    return hipGetLastError();
}

// Automatic launch shape, from measurements on MI355X at 2^30 draws over
// 262,144 streams (interleaved medians):
//   f64 uniforms   2 streams/lane (16-byte stores), ~2 waves per SIMD, each
//                  stream whole in one work-item, 512 threads whose waves
//                  pass a barrier per row (1.31 ms against 1.52 ms for the
//                  same grid running free), XCD remap
//   f32/u32        4 streams/lane, ~4 waves per SIMD, 512 threads, no remap
//                  (VALU-bound: the per-row barrier costs ~5%)
//   exponential    2 streams/lane, ~4 waves per SIMD (2 chunks per stream),
//                  256 threads, XCD remap
//   normal         2 streams/lane, ~8 waves per SIMD (flat from 2 to 16),
//                  256 threads, XCD remap
// Chunks hold at least 96 units (32 with one stream per lane on grids below
// two waves per SIMD); at most 65535 chunks.  A narrower store is used when n_streams or the output
// alignment does not allow the wide one.
// Index of the tuned shape for a call: kind (dist, dtype) and size class of
// its draw count.
static const TunedShape& tuned_shape(const GenLaunch& L) {
    int kind;
    switch (L.dist) {
        case kUniform: kind = L.dtype == kF64 ? 0 : 1; break;
        case kRaw: kind = 2; break;
        case kNormal: kind = L.dtype == kF64 ? 3 : 4; break;
        default: kind = L.dtype == kF64 ? 5 : 6; break;
    }
    const uint64_t n = L.q * L.S + L.r;
    const int cls = n < (1ull << 18) ? 0 : n < (1ull << 22) ? 1 : n < (1ull << 26) ? 2 : n < (1ull << 29) ? 3 : 4;
    return kTuned[kind][cls];
}

void plan_generate(GenLaunch& L) {
    const int esz = L.dtype == kF64 ? 8 : 4;
    const TunedShape& t = tuned_shape(L);
    const bool cfg_given = L.block || L.chunk || L.spl || (L.arith && L.arith != kArith31);
    if (!L.arith) L.arith = kArithF64;
    const bool spl_auto = !L.spl;
    if (spl_auto) L.spl = t.spl;
    if (!L.block) L.block = t.block;
    if (!cfg_given) {
        // Non-temporal stores when rows start on 128-byte lines; otherwise
        // the line a wave shares with its neighbour is written in two halves,
        // which L2 merges only when it keeps them (2^30 fp64 uniforms over
        // 262,143 streams: 2.13 ms with nt stores, 1.80 ms without)
        L.nontemporal = (static_cast<uint64_t>(L.S) * esz) % 128 == 0;
        L.xcd = t.xcd;
    }
    // at most 16 bytes per store; narrower when the shape does not allow it
    while (L.spl * esz > 16) L.spl /= 2;
    while (L.spl > 1 && (L.S % L.spl || reinterpret_cast<uintptr_t>(L.out) % (L.spl * esz))) L.spl /= 2;
    if (spl_auto)  // fewer streams than a wave would cover: lanes would idle
        while (L.spl > 1 && 64ull * L.spl > L.S) L.spl /= 2;
    const uint64_t cnt_max = L.q + (L.r ? 1 : 0);
    const uint64_t units_max = L.dist == kNormal ? (cnt_max + 1) / 2 : cnt_max;
    const uint64_t n_sblk = (static_cast<uint64_t>(L.S) + 64ull * L.spl - 1) / (64ull * L.spl);
    if (!L.chunk) {
        // chunk for about t.waves waves, at least t.min_units units each
        uint64_t w = (t.waves + n_sblk - 1) / n_sblk;
        const uint64_t w_cap = (units_max + t.min_units - 1) / t.min_units;
        if (w > w_cap) w = w_cap;
        if (w < 1) w = 1;
        const uint64_t c = (units_max + w - 1) / w;
        L.chunk = static_cast<uint32_t>(c > 0xffffffffull ? 0xffffffffull : (c ? c : 1));
    }
    uint64_t nch = units_max ? (units_max + L.chunk - 1) / L.chunk : 0;
    if (nch > 65535) {
        uint64_t c = (units_max + 65534) / 65535;
        L.chunk = static_cast<uint32_t>(c);
        nch = (units_max + c - 1) / c;
    }
    L.n_chunks = static_cast<uint32_t>(nch);
    // Lockstep rows (store-bound fp64 uniforms): once the grid fills the
    // chip (two waves per SIMD), the waves of a block writing each row
    // together beat free-running waves; smaller grids are launch-latency-bound
    if (!cfg_given && t.lock) L.lock = n_sblk * nch >= 2048;
    const uint64_t wpb = static_cast<uint64_t>(L.block) / 64;
    const uint64_t gx = (n_sblk + wpb - 1) / wpb;
    if (L.xcd && (gx * nch) % 8) L.xcd = 0;  // the remap needs a multiple of 8 blocks
}

template <int DIST, int DTYPE, int ARITH, int SPL, bool NT, bool LOCK>
static hipError_t launch_t(const GenLaunch& L, hipStream_t s) {
    const unsigned wpb = static_cast<unsigned>(L.block) / 64;
    const uint64_t ws = 64ull * SPL;
    const uint64_t n_sblk = (static_cast<uint64_t>(L.S) + ws - 1) / ws;
    dim3 grid(static_cast<unsigned>((n_sblk + wpb - 1) / wpb), L.n_chunks);
    hipLaunchKernelGGL((gen_kernel<DIST, DTYPE, ARITH, SPL, NT, LOCK>), grid, dim3(L.block), 0, s, L);
    return hipGetLastError();
}

template <int DIST, int DTYPE, int ARITH, int SPL>
static hipError_t launch_nt(const GenLaunch& L, hipStream_t s) {
    if (L.nontemporal)
        return L.lock ? launch_t<DIST, DTYPE, ARITH, SPL, true, true>(L, s)
                      : launch_t<DIST, DTYPE, ARITH, SPL, true, false>(L, s);
    return L.lock ? launch_t<DIST, DTYPE, ARITH, SPL, false, true>(L, s)
                  : launch_t<DIST, DTYPE, ARITH, SPL, false, false>(L, s);
}

template <int DIST, int DTYPE, int ARITH>
static hipError_t launch_spl(const GenLaunch& L, hipStream_t s) {
    if constexpr (DTYPE == kF64) {
        if (L.spl == 2) return launch_nt<DIST, DTYPE, ARITH, 2>(L, s);
    } else {
        if (L.spl == 4) return launch_nt<DIST, DTYPE, ARITH, 4>(L, s);
        if (L.spl == 2) return launch_nt<DIST, DTYPE, ARITH, 2>(L, s);
    }
    return launch_nt<DIST, DTYPE, ARITH, 1>(L, s);
}

template <int DIST, int DTYPE>
static hipError_t launch_dd(const GenLaunch& L, hipStream_t s) {
    if (L.arith == kArith31) return launch_spl<DIST, DTYPE, kArith31>(L, s);
    if (L.arith == kArithF64) return launch_spl<DIST, DTYPE, kArithF64>(L, s);
    return launch_spl<DIST, DTYPE, kArithInt>(L, s);
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

// ------------------------------------------------------ store-only ceiling
// The store pattern of gen_kernel for uniforms (same block -> (stream block,
// chunk) map, XCD remap, per-lane store width, row order, per-row barriers
// and cache policy) with a constant in place of the numbers: its time is
// what the layout allows the writes alone.  Full rows only (n a multiple of
// S, checked by the caller).
template <typename T, int SPL, bool NT, bool LOCK>
__global__ void __launch_bounds__(1024) store_ceiling_kernel(GenLaunch L, T value) {
    uint32_t bx = blockIdx.x, by = blockIdx.y;
    if (L.xcd) {
        const uint32_t total = gridDim.x * gridDim.y;
        uint32_t lin = blockIdx.x + blockIdx.y * gridDim.x;
        lin = (lin % 8) * (total / 8) + lin / 8;
        bx = lin % gridDim.x;
        by = lin / gridDim.x;
    }
    constexpr uint32_t ESZ = sizeof(T);
    constexpr uint32_t WS = 64 * SPL;
    const uint32_t wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const uint32_t sblk = bx * (blockDim.x >> 6) + wave;
    const bool live = sblk < (L.S + WS - 1) / WS;
    if (!LOCK && !live) return;
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t first = sblk * WS;
    const bool mine = live && first + lane * SPL < L.S;
    const uint64_t u0 = static_cast<uint64_t>(by) * L.chunk;
    const uint64_t u1 = min(u0 + L.chunk, L.q);
    const uint64_t rowstep = static_cast<uint64_t>(L.S) * ESZ;
    const uint64_t rest = live ? static_cast<uint64_t>(L.S - first) * ESZ : 0;
    const uint32_t nrec = rest > 0xffffffffull ? 0xffffffffu : static_cast<uint32_t>(rest);
    const uint32_t voff = lane * SPL * ESZ;
    const char* row = static_cast<const char*>(L.out) + (u0 * L.S + (live ? first : 0)) * ESZ;
    Pack<T, SPL> p;
#pragma unroll
    for (int i = 0; i < SPL; ++i) p.v[i] = value;
    for (uint64_t k = u0; k < u1; ++k) {
        if (mine) store_n<T, SPL, NT>(row_rsrc(row, nrec), voff, p);
        row += rowstep;
        if constexpr (LOCK) __builtin_amdgcn_s_barrier();
    }
}

template <typename T, int SPL>
static hipError_t launch_ceiling_t(const GenLaunch& L, T value, hipStream_t s) {
    const unsigned wpb = static_cast<unsigned>(L.block) / 64;
    const uint64_t n_sblk = (static_cast<uint64_t>(L.S) + 64 * SPL - 1) / (64 * SPL);
    dim3 grid(static_cast<unsigned>((n_sblk + wpb - 1) / wpb), L.n_chunks);
    if (L.nontemporal) {
        if (L.lock) hipLaunchKernelGGL((store_ceiling_kernel<T, SPL, true, true>), grid, dim3(L.block), 0, s, L, value);
        else hipLaunchKernelGGL((store_ceiling_kernel<T, SPL, true, false>), grid, dim3(L.block), 0, s, L, value);
    } else {
        if (L.lock) hipLaunchKernelGGL((store_ceiling_kernel<T, SPL, false, true>), grid, dim3(L.block), 0, s, L, value);
        else hipLaunchKernelGGL((store_ceiling_kernel<T, SPL, false, false>), grid, dim3(L.block), 0, s, L, value);
    }
    return hipGetLastError();
}

hipError_t launch_store_ceiling(const GenLaunch& L, hipStream_t s) {
    if (L.n_chunks == 0) return hipSuccess;
    if (L.dtype == kF64) {
        if (L.spl == 2) return launch_ceiling_t<double, 2>(L, 0.5, s);
        return launch_ceiling_t<double, 1>(L, 0.5, s);
    }
    if (L.spl == 4) return launch_ceiling_t<float, 4>(L, 0.5f, s);
    if (L.spl == 2) return launch_ceiling_t<float, 2>(L, 0.5f, s);
    return launch_ceiling_t<float, 1>(L, 0.5f, s);
}

int batch_gang_blocks_per_cu(unsigned block, bool narrow) {
    static std::mutex mu;
    static int cached[2][9] = {};  // by kernel and waves per block
    const unsigned w = block / 64;
    if (w == 0 || w > 8) return 1;
    std::lock_guard<std::mutex> lk(mu);
    int& c = cached[narrow ? 1 : 0][w];
    if (!c) {
        const void* k = narrow ? reinterpret_cast<const void*>(batch_gang_narrow_kernel)
                               : reinterpret_cast<const void*>(batch_gang_kernel);
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, static_cast<int>(block), 0) != hipSuccess || n <= 0)
            n = 1;
        c = n;
    }
    return c;
}

int batch_kind(int dist, int dtype, int spl) {
    switch (dist) {
        case kUniform:
            if (dtype == kF64) return spl == 2 ? kBUniF64x2 : kBUniF64x1;
            return spl == 4 ? kBUniF32x4 : kBUniF32x1;
        case kRaw: return spl == 4 ? kBRawU32x4 : kBRawU32x1;
        case kNormal:
            if (spl == 2) return dtype == kF64 ? kBNormF64x2 : kBNormF32x2;
            return dtype == kF64 ? kBNormF64 : kBNormF32;
        default:
            if (spl == 2) return dtype == kF64 ? kBExpF64x2 : kBExpF32x2;
            return dtype == kF64 ? kBExpF64 : kBExpF32;
    }
}

// Blocks of the persistent batch kernel that fit on one CU at once (a
// property of the compiled kernel; computed once, thread-safely).
int batch_blocks_per_cu() {
    static const int cached = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, reinterpret_cast<const void*>(batch_kernel), 256, 0) !=
                hipSuccess || n <= 0)
            n = 1;
        return n;
    }();
    return cached;
}

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0)
        return 256;
    return cus;
}

hipError_t launch_batch(const BatchLaunch& B_in, unsigned grid, unsigned block, hipStream_t s) {
    BatchLaunch B = B_in;
    B.wpb = block / 64;
    B.grid = grid;
    hipLaunchKernelGGL(batch_init_kernel, dim3(grid1d(B.n_req ? B.n_req : 1, 256)), dim3(256), 0, s, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (B.n_gangs && B.narrow) hipLaunchKernelGGL(batch_gang_narrow_kernel, dim3(grid), dim3(block), 0, s, B);
    else if (B.n_gangs) hipLaunchKernelGGL(batch_gang_kernel, dim3(grid), dim3(block), 0, s, B);
    else hipLaunchKernelGGL(batch_kernel, dim3(grid), dim3(block), 0, s, B);
    e = hipGetLastError();
    if (e != hipSuccess || B.fin_total == 0) return e;
    hipLaunchKernelGGL(batch_finalize_kernel, dim3(static_cast<unsigned>((B.fin_total + 255) / 256)),
                       dim3(256), 0, s, B);
    return hipGetLastError();
}

hipError_t launch_generate(const GenLaunch& L, hipStream_t s) {
    if (L.n_chunks == 0) return hipSuccess;
    hipError_t e = launch_gen_only(L, s);
    if (e != hipSuccess || L.n_chunks == 1 || L.no_writeback) return e;
    if (L.arith == kArith31)
        hipLaunchKernelGGL(finalize_kernel<kGen31k3p>, dim3(grid1d(L.S, 256)), dim3(256), 0, s, L.streams, L.S,
                           L.q, L.r, L.dist == kNormal ? 1 : 0);
    else
        hipLaunchKernelGGL(finalize_kernel<kGen32k3a>, dim3(grid1d(L.S, 256)), dim3(256), 0, s, L.streams, L.S,
                           L.q, L.r, L.dist == kNormal ? 1 : 0);
    return hipGetLastError();
}

// ------------------------------------------------- the paper's geometry
// Listing 1 (Section 2.2) and Listing 2 (Section 3.1): a G0 x G1 lattice of
// work-items; work-item (g0, g1) owns the cells (g0 + i G0, g1 + j G1) of
// the nrow x ncol output (row stride npad) and visits them row by row.  Its
// stream is g0 + G0 g1 for uniforms and integers, g0 G1 + g1 for normals and
// exponentials.  Normals pair the work-items (g0, 2p) and (g0, 2p+1): one
// lane runs both streams, U1 from the first, U2 from the second, X and Y to
// the two adjacent cells.
//
// A lane runs one work-item (or pair) over a chunk of its visits: a block of
// its rows, or, where a work-item has fewer rows than the chunks wanted, a
// block of one row's visits.  Lanes with neighbouring g1 write neighbouring
// columns of the same rows in step.  The lane jumps its stream(s) to the
// chunk's first visit; with one chunk per work-item it writes the state back,
// otherwise paper_finalize_kernel does, after the launch.
template <int G>
struct EngineOf {
    using T = F64Engine;
};
template <>
struct EngineOf<kGen31k3p> {
    using T = Engine31;
};

__device__ __forceinline__ uint64_t paper_stream_of(int dist, uint32_t g0, uint32_t g1, uint32_t G0, uint32_t G1) {
    return (dist == kUniform || dist == kRaw) ? g0 + static_cast<uint64_t>(G0) * g1
                                              : static_cast<uint64_t>(g0) * G1 + g1;
}

// Advance a stream record by e steps (e wave-uniform) by the fp64 digit tables.
template <int G>
__device__ __forceinline__ void paper_jump(uint32_t x[6], uint64_t e) {
    dev_jump_digits<G>(x, e);
}

__host__ __device__ inline uint64_t paper_lanes_per_chunk(const PaperLaunch& L) {
    return (static_cast<uint64_t>(L.G0) * L.lanes_g1 + 63) / 64 * 64;
}

template <int DIST, int DTYPE, int G>
__global__ void __launch_bounds__(256) paper_kernel(PaperLaunch L) {
    if constexpr (DIST == kNormal || DIST == kExponential) stage_tables();
    using Engine = typename EngineOf<G>::T;
    using T = typename ElemOf<DTYPE>::T;
    const uint64_t id = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    // lanes per chunk, a whole number of waves: every wave lies in one chunk,
    // so the chunk and its jump exponents are wave-uniform (scalar table reads)
    const uint64_t per_chunk = paper_lanes_per_chunk(L);
    if (id >= per_chunk * L.n_rb * L.n_cb) return;
    const uint32_t ch = __builtin_amdgcn_readfirstlane(static_cast<uint32_t>(id / per_chunk));
    const uint32_t rb = ch / L.n_cb, cb = ch % L.n_cb;
    const uint64_t rem = id % per_chunk;
    if (rem >= static_cast<uint64_t>(L.G0) * L.lanes_g1) return;  // padding of the last wave
    const uint32_t g0 = static_cast<uint32_t>(rem / L.lanes_g1);
    const uint32_t h = static_cast<uint32_t>(rem % L.lanes_g1);
    const uint32_t g1 = DIST == kNormal ? 2 * h : h;
    if (g0 >= L.nrow || g1 >= L.ncol) return;  // the work-item owns no cell
    const uint32_t nr = (L.nrow - 1 - g0) / L.G0 + 1;
    const uint32_t nc = (L.ncol - 1 - g1) / L.G1 + 1;
    const uint32_t nc_max = (L.ncol - 1) / L.G1 + 1;  // nc is nc_max or nc_max - 1
    const uint32_t i0 = rb * L.rows_per, j0 = cb * L.cols_per;
    if (i0 >= nr || j0 >= nc) return;
    const uint32_t i1 = min(nr, i0 + L.rows_per), j1 = min(nc, j0 + L.cols_per);

    // visits before the chunk: i0 nc + j0 = [i0 (nc_max - 1) + j0] + [i0 if nc == nc_max],
    // two jumps with wave-uniform exponents
    const uint64_t e_all = static_cast<uint64_t>(i0) * (nc_max - 1) + j0;
    const bool longer = nc == nc_max && i0 > 0;
    uint32_t* ra = L.streams + paper_stream_of(DIST, g0, g1, L.G0, L.G1) * 18;
    uint32_t* rb_rec = DIST == kNormal ? L.streams + paper_stream_of(DIST, g0, g1 + 1, L.G0, L.G1) * 18 : ra;
    uint32_t x[6];
    Engine ea, eb;
#pragma unroll
    for (int w = 0; w < 6; ++w) x[w] = ra[w];
    if (e_all) paper_jump<G>(x, e_all);
    if (longer) paper_jump<G>(x, i0);
    ea.load(x);
    if constexpr (DIST == kNormal) {
#pragma unroll
        for (int w = 0; w < 6; ++w) x[w] = rb_rec[w];
        if (e_all) paper_jump<G>(x, e_all);
        if (longer) paper_jump<G>(x, i0);
        eb.load(x);
    }
    T* out = static_cast<T*>(L.out);
    const double inv_rate = L.param;
    for (uint32_t i = i0; i < i1; ++i) {
        T* row = out + (g0 + static_cast<uint64_t>(i) * L.G0) * L.npad;
        for (uint32_t j = j0, c = g1 + j0 * L.G1; j < j1; ++j, c += L.G1) {
            if constexpr (DIST == kNormal) {
                auto z1 = ea.step_rot();
                auto z2 = eb.step_rot();
                double xv, yv;
                box_muller<G, DTYPE>(z1, z2, xv, yv);
                __builtin_nontemporal_store(narrow<DTYPE>(xv), row + c);
                __builtin_nontemporal_store(narrow<DTYPE>(yv), row + c + 1);
            } else {
                __builtin_nontemporal_store(value1<DIST, DTYPE, G>(ea.step_rot(), inv_rate), row + c);
            }
        }
        if (L.n_cb > 1) break;  // a column block covers one row
    }
    if (L.n_rb == 1 && L.n_cb == 1) {
        ea.save(x);
#pragma unroll
        for (int w = 0; w < 6; ++w) ra[w] = x[w];
        if constexpr (DIST == kNormal) {
            eb.save(x);
#pragma unroll
            for (int w = 0; w < 6; ++w) rb_rec[w] = x[w];
        }
    }
}

// After a launch with several chunks per work-item: every used stream
// advances by its work-item's number of visits.
template <int G>
__global__ void __launch_bounds__(256) paper_finalize_kernel(PaperLaunch L) {
    const uint64_t id = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (id >= static_cast<uint64_t>(L.G0) * L.lanes_g1) return;
    const uint32_t g0 = static_cast<uint32_t>(id / L.lanes_g1);
    const uint32_t h = static_cast<uint32_t>(id % L.lanes_g1);
    const bool normal = L.dist == kNormal;
    const uint32_t g1 = normal ? 2 * h : h;
    if (g0 >= L.nrow || g1 >= L.ncol) return;
    const uint64_t visits = static_cast<uint64_t>((L.nrow - 1 - g0) / L.G0 + 1) * ((L.ncol - 1 - g1) / L.G1 + 1);
    for (int k = 0; k < (normal ? 2 : 1); ++k) {
        uint32_t* rec = L.streams + paper_stream_of(L.dist, g0, g1 + k, L.G0, L.G1) * 18;
        uint32_t x[6];
#pragma unroll
        for (int w = 0; w < 6; ++w) x[w] = rec[w];
        dev_jump_digits<G>(x, visits);
#pragma unroll
        for (int w = 0; w < 6; ++w) rec[w] = x[w];
    }
}

template <int DIST, int DTYPE, int G>
static int paper_blocks_per_cu() {
    static const int cached = [] {
        int n = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
                &n, reinterpret_cast<const void*>(paper_kernel<DIST, DTYPE, G>), 256, 0) != hipSuccess || n <= 0)
            n = 1;
        return n;
    }();
    return cached;
}

template <int G>
static int paper_blocks_per_cu_g(int dist, int dtype) {
    switch (dist) {
        case kUniform: return dtype == kF64 ? paper_blocks_per_cu<kUniform, kF64, G>()
                                            : paper_blocks_per_cu<kUniform, kF32, G>();
        case kNormal: return dtype == kF64 ? paper_blocks_per_cu<kNormal, kF64, G>()
                                           : paper_blocks_per_cu<kNormal, kF32, G>();
        case kExponential: return dtype == kF64 ? paper_blocks_per_cu<kExponential, kF64, G>()
                                                : paper_blocks_per_cu<kExponential, kF32, G>();
        default: return paper_blocks_per_cu<kRaw, kU32, G>();
    }
}

// Chunks per work-item: about as many as fill a whole number of rounds of
// the waves the device holds at once -- one for normals and exponentials, so
// that every lane runs one chunk of about equal length and no partly filled
// round trails the launch, three for uniforms and raw words, whose stores
// keep more waves busy over time -- in whole rows while a work-item has
// enough of them, else in blocks of one row's visits.  The 10^4 x 10^4
// normals of Section 3.1 on a 512 x 128 lattice (32,768 pairs, 20 rows of
// 78-79 visits each): 0.29 ms against 0.41 ms in one-row blocks for 2^20
// lanes with per-bit jumps; fp64 uniforms 0.165 against 0.18 ms.
#ifndef MRG_PAPER_ROUNDS
#define MRG_PAPER_ROUNDS 1
#endif
#ifndef MRG_PAPER_ROUNDS_PLAIN
#define MRG_PAPER_ROUNDS_PLAIN 3
#endif
constexpr uint64_t kPaperRounds = MRG_PAPER_ROUNDS;             // normals, exponentials
constexpr uint64_t kPaperRoundsPlain = MRG_PAPER_ROUNDS_PLAIN;  // uniforms, raw (store-bound)

void plan_paper(PaperLaunch& L, int gen) {
    L.lanes_g1 = L.dist == kNormal ? L.G1 / 2 : L.G1;
    const uint64_t nr_max = (static_cast<uint64_t>(L.nrow) + L.G0 - 1) / L.G0;
    const uint64_t nc_max = (static_cast<uint64_t>(L.ncol) + L.G1 - 1) / L.G1;
    const uint64_t items = paper_lanes_per_chunk(L);
    const int per_cu = gen == kGen31k3p ? paper_blocks_per_cu_g<kGen31k3p>(L.dist, L.dtype)
                                        : paper_blocks_per_cu_g<kGen32k3a>(L.dist, L.dtype);
    const uint64_t resident = static_cast<uint64_t>(device_cu_count()) * static_cast<uint64_t>(per_cu) * 256;
    const uint64_t rounds = L.dist == kUniform || L.dist == kRaw ? kPaperRoundsPlain : kPaperRounds;
    const uint64_t want = std::max<uint64_t>(1, rounds * resident / std::max<uint64_t>(1, items));
    if (want <= nr_max || nc_max <= 1) {
        L.rows_per = static_cast<uint32_t>((nr_max + want - 1) / want);
        if (L.rows_per == 0) L.rows_per = 1;
        L.n_rb = static_cast<uint32_t>((nr_max + L.rows_per - 1) / L.rows_per);
        L.cols_per = static_cast<uint32_t>(nc_max);
        L.n_cb = 1;
    } else {
        L.rows_per = 1;
        L.n_rb = static_cast<uint32_t>(nr_max);
        const uint64_t per_row = std::min<uint64_t>(nc_max, (want + nr_max - 1) / nr_max);
        L.cols_per = static_cast<uint32_t>((nc_max + per_row - 1) / per_row);
        L.n_cb = static_cast<uint32_t>((nc_max + L.cols_per - 1) / L.cols_per);
    }
    if (L.n_rb == 0) L.n_rb = 1;
    if (L.n_cb == 0) L.n_cb = 1;
}

template <int DIST, int DTYPE>
static hipError_t launch_paper_t(const PaperLaunch& L, int gen, hipStream_t s) {
    const uint64_t lanes = paper_lanes_per_chunk(L) * L.n_rb * L.n_cb;
    const dim3 grid(static_cast<unsigned>((lanes + 255) / 256));
    if (gen == kGen32k3a) hipLaunchKernelGGL((paper_kernel<DIST, DTYPE, kGen32k3a>), grid, dim3(256), 0, s, L);
    else hipLaunchKernelGGL((paper_kernel<DIST, DTYPE, kGen31k3p>), grid, dim3(256), 0, s, L);
    return hipGetLastError();
}

hipError_t launch_paper(const PaperLaunch& L, int gen, hipStream_t s) {
    hipError_t e;
    switch (L.dist) {
        case kUniform:
            e = L.dtype == kF64 ? launch_paper_t<kUniform, kF64>(L, gen, s) : launch_paper_t<kUniform, kF32>(L, gen, s);
            break;
        case kNormal:
            e = L.dtype == kF64 ? launch_paper_t<kNormal, kF64>(L, gen, s) : launch_paper_t<kNormal, kF32>(L, gen, s);
            break;
        case kExponential:
            e = L.dtype == kF64 ? launch_paper_t<kExponential, kF64>(L, gen, s)
                                : launch_paper_t<kExponential, kF32>(L, gen, s);
            break;
        default:
            e = launch_paper_t<kRaw, kU32>(L, gen, s);
    }
    if (e != hipSuccess || (L.n_rb == 1 && L.n_cb == 1)) return e;
    const uint64_t items = static_cast<uint64_t>(L.G0) * L.lanes_g1;
    const dim3 grid(static_cast<unsigned>((items + 255) / 256));
    if (gen == kGen32k3a) hipLaunchKernelGGL(paper_finalize_kernel<kGen32k3a>, grid, dim3(256), 0, s, L);
    else hipLaunchKernelGGL(paper_finalize_kernel<kGen31k3p>, grid, dim3(256), 0, s, L);
    return hipGetLastError();
}

}  // namespace mrg355
