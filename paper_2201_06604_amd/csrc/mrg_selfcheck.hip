// mrg_selfcheck.hip -- diagnostics: the library's own transcendentals against
// the HIP device math library over whole input ranges.
//
// The normal and exponential transforms use log_unit, sqrt_radius and
// sincospi_unit (mrg_engine.h) instead of the general library functions:
// they leave out range reduction and special cases that the generators'
// uniforms can never reach.  mrg_transform_accuracy evaluates one of them and
// the library function on every integer z of a range -- the input each
// generator step can produce -- and histograms the distance in units in the
// last place, so that a caller can check the whole input domain (2^32 values)
// in a few milliseconds.
#include <hip/hip_runtime.h>

#include "mrg355.h"
#include "mrg_engine.h"
#include "mrg_internal.h"
#include "mrg_math.h"

namespace mrg355 {

// Doubles mapped to integers that increase with the value (+0 and -0 both
// map to 0), so that the difference of two mapped values counts the
// representable doubles between them.
__device__ __forceinline__ int64_t ordered(double x) {
    const int64_t b = __double_as_longlong(x);
    return b >= 0 ? b : static_cast<int64_t>(0x8000000000000000ull) - b;
}

__device__ __forceinline__ uint64_t ulp_distance(double a, double b) {
    const int64_t d = ordered(a) - ordered(b);
    return static_cast<uint64_t>(d < 0 ? -d : d);
}

template <int G>
__device__ __forceinline__ uint64_t distance_at(int fn, uint64_t z) {
    constexpr double norm = G == kGen32k3a ? kNorm : kNorm31;
    const double u = static_cast<double>(z) * norm;
    if (fn == MRG_CHECK_LOG) return ulp_distance(log_unit(u), log(u));
    if (fn == MRG_CHECK_LOG_F32OUT) return ulp_distance(log_unit_f32out(u), log(u));
    if (fn == MRG_CHECK_SQRT || fn == MRG_CHECK_SQRT_F32OUT) {
        const double x = log_unit<-2>(u);  // the Box-Muller radius argument
        return ulp_distance(fn == MRG_CHECK_SQRT ? sqrt_radius(x) : sqrt_radius_f32out(x), sqrt(x));
    }
    // the Box-Muller angle argument 2u, formed as the kernels form it
    const double t = static_cast<double>(z) * (2.0 * norm);
    double s, c, s_ref, c_ref;
    if (fn == MRG_CHECK_SINPI || fn == MRG_CHECK_COSPI) sincospi_unit(t, &s, &c);
    else sincospi_unit_f32out(t, &s, &c);
    sincospi(t, &s_ref, &c_ref);
    return (fn == MRG_CHECK_SINPI || fn == MRG_CHECK_SINPI_F32OUT) ? ulp_distance(s, s_ref) : ulp_distance(c, c_ref);
}

__global__ void __launch_bounds__(64) accuracy_clear_kernel(unsigned long long* res) {
    if (threadIdx.x < kAccuracyWords) res[threadIdx.x] = 0;
}

// Grid-stride over z in [z0, z1): per-lane counts, summed per block in LDS,
// then one atomic per block and word.  The largest distance is packed as
// (distance << 32) | z, so an atomic maximum keeps the largest distance and,
// among equal ones, the largest z.
template <int G>
__global__ void __launch_bounds__(256) accuracy_kernel(int fn, uint64_t z0, uint64_t z1, unsigned long long* res) {
    stage_tables();
    __shared__ unsigned long long bins[kAccuracyBins];
    __shared__ unsigned long long worst;
    if (threadIdx.x < kAccuracyBins) bins[threadIdx.x] = 0;
    if (threadIdx.x == 0) worst = 0;
    __syncthreads();
    uint32_t cnt[kAccuracyBins] = {0, 0, 0, 0, 0};
    unsigned long long mine = 0;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    for (uint64_t z = z0 + static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x; z < z1; z += stride) {
        const uint64_t d = distance_at<G>(fn, z);
        const int bin = d < kAccuracyBins - 1 ? static_cast<int>(d) : kAccuracyBins - 1;
#pragma unroll
        for (int i = 0; i < kAccuracyBins; ++i) cnt[i] += bin == i ? 1u : 0u;
        const unsigned long long key = (static_cast<unsigned long long>(d < 0xffffffffull ? d : 0xffffffffull) << 32) | z;
        mine = key > mine ? key : mine;
    }
#pragma unroll
    for (int i = 0; i < kAccuracyBins; ++i)
        if (cnt[i]) atomicAdd(&bins[i], static_cast<unsigned long long>(cnt[i]));
    atomicMax(&worst, mine);
    __syncthreads();
    if (threadIdx.x < kAccuracyBins) atomicAdd(&res[threadIdx.x], bins[threadIdx.x]);
    if (threadIdx.x == 0) atomicMax(&res[kAccuracyBins], worst);
}

hipError_t launch_accuracy(int gen, int fn, uint64_t z0, uint64_t z1, unsigned long long* res, hipStream_t s) {
    hipLaunchKernelGGL(accuracy_clear_kernel, dim3(1), dim3(64), 0, s, res);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || z1 <= z0) return e;
    const uint64_t n = z1 - z0;
    const uint64_t want = (n + 256 * 64 - 1) / (256 * 64);  // about 64 inputs per lane at least
    const unsigned grid = static_cast<unsigned>(want < 8192 ? (want ? want : 1) : 8192);
    if (gen == kGen32k3a)
        hipLaunchKernelGGL(accuracy_kernel<kGen32k3a>, dim3(grid), dim3(256), 0, s, fn, z0, z1, res);
    else
        hipLaunchKernelGGL(accuracy_kernel<kGen31k3p>, dim3(grid), dim3(256), 0, s, fn, z0, z1, res);
    return hipGetLastError();
}

}  // namespace mrg355
