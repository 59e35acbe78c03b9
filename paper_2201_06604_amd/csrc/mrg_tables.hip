// mrg_tables.hip -- the Monte-Carlo Fisher test consumer of the streams
// (Section 4): random contingency tables with fixed margins, one stream per
// table, entries drawn in row-major order by inversion of their conditional
// hypergeometric distributions, one uniform per free entry.
//
// Each entry is sampled by hyper_invert_ck (mrg_hyper.h): the inversion that
// the oracle defines, with two shortcuts that give the same bits; the
// checkpoints of its search live in LDS.
//
// One lane owns one table.  The loops' trip counts depend on the margins, so
// lanes of a wave diverge; that is the price of exact inversion.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>
#include <vector>

#include "mrg_engine.h"
#include "mrg_hyper.h"
#include "mrg_internal.h"
#include "mrg_math.h"

namespace mrg355 {

// Inversion checkpoints per lane (LDS, 20 bytes each).  More shorten the
// second pass of a wide search but hold LDS that would otherwise let more
// blocks run: 10^6 tables of totals 5..200 took 2.27 / 2.25 / 2.12 / 2.06 /
// 2.39 ms with 3 / 4 / 5 / 6 / 8 (6: five blocks per CU); the paper's Fisher
// tables (totals about 12,900) 41.4 / 38.8 / 45.9 / 43.7 ms (Table 1) with
// 6 / 8 / 12 / 16.
#ifndef MRG_TABLE_CK
#define MRG_TABLE_CK 6
#endif
#ifndef MRG_FISHER_CK
#define MRG_FISHER_CK 8
#endif
constexpr int kTablesCk = MRG_TABLE_CK;
constexpr int kFisherCk = MRG_FISHER_CK;
constexpr int kTableBlock = 256;

// log(n!) for n <= kTableMaxTotal: lgamma(n+1) in long double on the host,
// rounded to double, uploaded once per device (ensure_logfact).  Every entry
// of a valid table is at most its grand total, so the index is in range.
__device__ double g_logfact[kTableMaxTotal + 1];

__device__ __forceinline__ double log_factorial(int n) { return g_logfact[n]; }

// One I x J table (I, J <= MAXD) with row totals r[], column totals c[]:
// entries to tab[i*ld + j] (when tab is not null); returns -sum log(n_ij!)
// summed row-major.  The engine advances (I-1)(J-1) steps.
template <int MAXD, int NCK, typename Engine>
__device__ double sample_table(Engine& e, double norm, int I, int J, const int32_t* r, const int32_t* c, int32_t* tab,
                               int ld, HyperCk ck) {
    int32_t crem[MAXD];
    for (int j = 0; j < J; ++j) crem[j] = c[j];
    double stat = 0.0;
    for (int i = 0; i < I - 1; ++i) {
        int64_t rrem = r[i];
        int64_t Np = 0;  // units left in columns j..J-1 over rows i..I-1
        for (int j = 0; j < J; ++j) Np += crem[j];
        for (int j = 0; j < J - 1; ++j) {
            const double u = to_f64(e.step_rot()) * norm;
            const int x = hyper_invert_ck<NCK>(u, Np, crem[j], rrem, ck);
            if (tab) tab[i * ld + j] = x;
            stat -= log_factorial(x);
            rrem -= x;
            Np -= crem[j];
            crem[j] -= x;
        }
        if (tab) tab[i * ld + J - 1] = static_cast<int32_t>(rrem);  // determined by the row total
        stat -= log_factorial(static_cast<int>(rrem));
        crem[J - 1] -= static_cast<int32_t>(rrem);
    }
    for (int j = 0; j < J; ++j) {  // the last row is what the columns have left
        if (tab) tab[(I - 1) * ld + j] = crem[j];
        stat -= log_factorial(crem[j]);
    }
    return stat;
}

// The engine and the scale 1/(m1+1) of generator G.
template <int G>
struct GenOf {
    using Engine = F64Engine;
    static constexpr double norm = kNorm;
};
template <>
struct GenOf<kGen31k3p> {
    using Engine = Engine31;
    static constexpr double norm = kNorm31;
};

// Table t: shape I[t] x J[t] (<= 5 x 5), margins rows[t][5], cols[t][5],
// from stream t; outputs tabs[t][5][5] (zero padded) and stats[t] (optional).
// A table whose shape is out of range or whose margins are negative, differ
// in total or total more than kTableMaxTotal gets zeros and a NaN statistic,
// and its stream is left as it was (the checks also bound every loop).
template <int G>
__device__ __forceinline__ void one_table(uint64_t t, uint32_t* streams, const int32_t* I, const int32_t* J,
                                          const int32_t* rows, const int32_t* cols, int32_t* tabs, double* stats,
                                          const HyperCk& ck) {
    int32_t* out = tabs + t * 25;
#pragma unroll
    for (int k = 0; k < 25; ++k) out[k] = 0;
    const int It = I[t], Jt = J[t];
    bool ok = It >= 1 && It <= 5 && Jt >= 1 && Jt <= 5;
    int64_t rs = 0, cs = 0;
    for (int k = 0; ok && k < It; ++k) {
        ok = rows[t * 5 + k] >= 0;
        rs += rows[t * 5 + k];
    }
    for (int k = 0; ok && k < Jt; ++k) {
        ok = cols[t * 5 + k] >= 0;
        cs += cols[t * 5 + k];
    }
    ok = ok && rs == cs && rs <= kTableMaxTotal;
    if (!ok) {
        if (stats) stats[t] = __builtin_nan("");
        return;
    }
    uint32_t* rec = streams + t * 18;
    uint32_t x[6];
#pragma unroll
    for (int w = 0; w < 6; ++w) x[w] = rec[w];
    typename GenOf<G>::Engine e;
    e.load(x);
    const double stat = sample_table<5, kTablesCk>(e, GenOf<G>::norm, It, Jt, rows + t * 5, cols + t * 5, out, 5, ck);
    if (stats) stats[t] = stat;
    e.save(x);
#pragma unroll
    for (int w = 0; w < 6; ++w) rec[w] = x[w];
}

// A block takes 256 consecutive tables.  A table makes (I-1)(J-1)
// inversions, 1 to 16, each searching a range that grows like the square
// root of the table's total, and a wave runs as long as its longest lane;
// so the block first orders its tables by the estimate (I-1)(J-1) sqrt(total)
// in 64 buckets (a counting sort in LDS: the order within a bucket does not
// matter, every table has its own stream and output), and each wave then
// takes 64 tables of about the same work (10^6 tables of the 2x2..5x5 mix:
// 2.62 -> 2.40 ms).  Sorting windows of 3 or 7 blocks' tables, taken in
// rounds by fewer blocks, were no faster or slower.
template <int G>
__global__ void __launch_bounds__(kTableBlock) tables_kernel(uint32_t* streams, uint64_t n, const int32_t* I,
                                                             const int32_t* J, const int32_t* rows, const int32_t* cols,
                                                             int32_t* tabs, double* stats) {
    __shared__ double ck_s[kTablesCk * kTableBlock], ck_w[kTablesCk * kTableBlock];
    __shared__ int ck_r[kTablesCk * kTableBlock];
    constexpr int kBuckets = 64;
    __shared__ uint16_t order[kTableBlock];
    __shared__ uint32_t start[kBuckets + 1];
    const HyperCk ck{ck_s + threadIdx.x, ck_w + threadIdx.x, ck_r + threadIdx.x, kTableBlock};
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kTableBlock;
    const uint32_t here = n - base < kTableBlock ? static_cast<uint32_t>(n - base) : kTableBlock;
    // bucket of the work estimate (0 for shapes out of range: they stop at once)
    auto key_of = [&](uint32_t k) {
        const uint64_t t = base + k;
        const int It = I[t], Jt = J[t];
        if (!(It >= 1 && It <= 5 && Jt >= 1 && Jt <= 5)) return 0u;
        int64_t total = 0;
        for (int r = 0; r < It; ++r) total += rows[t * 5 + r];
        const double est = (It - 1) * (Jt - 1) * __builtin_sqrt(static_cast<double>(total > 0 ? total : 0));
        const double b = est * 0.125;  // 16 inversions at a total of 1,000 reach bucket 63
        return b >= kBuckets - 1 ? static_cast<uint32_t>(kBuckets - 1) : static_cast<uint32_t>(b);
    };
    if (threadIdx.x <= kBuckets) start[threadIdx.x] = 0;
    __syncthreads();
    const uint32_t k = threadIdx.x;
    const uint32_t key = k < here ? key_of(k) : 0u;
    if (k < here) atomicAdd(&start[key + 1], 1u);
    __syncthreads();
    if (threadIdx.x == 0)
        for (int c = 1; c <= kBuckets; ++c) start[c] += start[c - 1];  // start[c] = tables in buckets below c
    __syncthreads();
    if (k < here) order[atomicAdd(&start[key], 1u)] = static_cast<uint16_t>(k);
    __syncthreads();
    if (k < here) one_table<G>(base + order[k], streams, I, J, rows, cols, tabs, stats, ck);
}

// The count is cleared by a kernel, not a memset, so the launch can be
// captured in a graph.
__global__ void fisher_clear_kernel(unsigned long long* count) { *count = 0; }

struct FisherArgs {
    uint32_t* streams;
    uint64_t B;
    int I, J;
    int32_t r[kFisherMaxDim], c[kFisherMaxDim];
    double threshold;      // observed statistic / (1 + 64 eps)
    unsigned long long* count;
    double* stats;
};

// Replicate b < B of the observed table's margins from stream b; counts the
// replicates whose statistic is <= threshold (one atomic per wave; every
// lane executes it, with the wave's count on lane 0 and 0 elsewhere).
template <int G>
__global__ void __launch_bounds__(kTableBlock) fisher_kernel(FisherArgs a) {
    __shared__ double ck_s[kFisherCk * kTableBlock], ck_w[kFisherCk * kTableBlock];
    __shared__ int ck_r[kFisherCk * kTableBlock];
    const HyperCk ck{ck_s + threadIdx.x, ck_w + threadIdx.x, ck_r + threadIdx.x, kTableBlock};
    const uint64_t b = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63;
    bool hit = false;
    if (b < a.B) {
        uint32_t* rec = a.streams + b * 18;
        uint32_t x[6];
#pragma unroll
        for (int w = 0; w < 6; ++w) x[w] = rec[w];
        typename GenOf<G>::Engine e;
        e.load(x);
        const double stat =
            sample_table<kFisherMaxDim, kFisherCk>(e, GenOf<G>::norm, a.I, a.J, a.r, a.c, nullptr, 0, ck);
        hit = stat <= a.threshold;
        if (a.stats) a.stats[b] = stat;
        e.save(x);
#pragma unroll
        for (int w = 0; w < 6; ++w) rec[w] = x[w];
    }
    const unsigned long long wave_hits = __popcll(__ballot(hit));
    atomicAdd(a.count, lane == 0 ? wave_hits : 0ull);
}

double host_log_factorial(int64_t k) {
    int sign = 0;
    return static_cast<double>(lgammal_r(static_cast<long double>(k) + 1.0L, &sign));
}

// One upload of the log-factorial table per device, before the first table
// launch there (synchronous; a launch captured in a graph needs one call
// made beforehand on the device).
hipError_t ensure_logfact() {
    static std::mutex mu;
    static std::vector<char> ready;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    std::lock_guard<std::mutex> lk(mu);
    if (static_cast<size_t>(dev) < ready.size() && ready[dev]) return hipSuccess;
    static std::vector<double> host;
    if (host.empty()) {
        host.resize(kTableMaxTotal + 1);
        for (int64_t k = 0; k <= kTableMaxTotal; ++k)
            host[k] = host_log_factorial(k);
    }
    e = hipMemcpyToSymbol(HIP_SYMBOL(g_logfact), host.data(), host.size() * sizeof(double));
    if (e != hipSuccess) return e;
    if (ready.size() <= static_cast<size_t>(dev)) ready.resize(dev + 1, 0);
    ready[dev] = 1;
    return hipSuccess;
}

hipError_t launch_tables(int gen, uint32_t* streams, uint64_t n, const int32_t* I, const int32_t* J,
                         const int32_t* rows, const int32_t* cols, int32_t* tabs, double* stats, hipStream_t s) {
    if (hipError_t e = ensure_logfact()) return e;
    const dim3 grid(static_cast<unsigned>((n + kTableBlock - 1) / kTableBlock));
    if (gen == kGen32k3a)
        hipLaunchKernelGGL(tables_kernel<kGen32k3a>, grid, dim3(kTableBlock), 0, s, streams, n, I, J, rows, cols, tabs,
                           stats);
    else
        hipLaunchKernelGGL(tables_kernel<kGen31k3p>, grid, dim3(kTableBlock), 0, s, streams, n, I, J, rows, cols, tabs,
                           stats);
    return hipGetLastError();
}

hipError_t launch_fisher(int gen, uint32_t* streams, uint64_t B, int I, int J, const int32_t* r, const int32_t* c,
                         double threshold, unsigned long long* count, double* stats, hipStream_t s) {
    FisherArgs a{};
    a.streams = streams;
    a.B = B;
    a.I = I;
    a.J = J;
    for (int k = 0; k < kFisherMaxDim; ++k) {
        a.r[k] = k < I ? r[k] : 0;
        a.c[k] = k < J ? c[k] : 0;
    }
    a.threshold = threshold;
    a.count = count;
    a.stats = stats;
    if (B) {
        if (hipError_t e = ensure_logfact()) return e;
    }
    hipLaunchKernelGGL(fisher_clear_kernel, dim3(1), dim3(1), 0, s, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || B == 0) return e;
    const dim3 grid(static_cast<unsigned>((B + kTableBlock - 1) / kTableBlock));
    if (gen == kGen32k3a) hipLaunchKernelGGL(fisher_kernel<kGen32k3a>, grid, dim3(kTableBlock), 0, s, a);
    else hipLaunchKernelGGL(fisher_kernel<kGen31k3p>, grid, dim3(kTableBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace mrg355
