// mrg_internal.h -- interface between the C-ABI layer (mrg_api.cpp) and the
// gfx950 kernels (mrg_kernels.hip).  Not installed; not part of the ABI.
#pragma once

#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace mrg355 {

enum Dist { kUniform = 0, kNormal = 1, kExponential = 2, kRaw = 3 };
enum DType { kF64 = 0, kF32 = 1, kU32 = 2 };
enum Arith { kArithAuto = 0, kArithInt = 1, kArithF64 = 2 };

// One plain generation launch over S streams (see mrg_generate).
struct GenLaunch {
    uint32_t* streams;   // S records of 18 words; `cur` is read and written
    void* out;           // dense n elements
    uint64_t q;          // floor(n / S)
    uint32_t S;          // streams
    uint32_t r;          // n mod S
    uint32_t chunk;      // units (draws; normal: pairs) per work-item
    uint32_t n_chunks;   // work-items per stream
    double param;        // 1/rate for exponentials
    int dist, dtype, arith, block, nontemporal;
    int spl;             // streams per lane (1, 2, 4); 0 = automatic
    int xcd;             // 1 = XCD-contiguous block order
};

// Resolve chunk/n_chunks/block/arith left at 0 to the automatic choice.
void plan_generate(GenLaunch& L);
hipError_t launch_generate(const GenLaunch& L, hipStream_t s);

hipError_t launch_create(uint32_t* out, uint64_t n, const uint32_t creator[6], hipStream_t s);
hipError_t launch_reset(uint32_t* streams, uint64_t n, int kind, hipStream_t s);
hipError_t launch_advance(uint32_t* streams, uint64_t n, uint64_t steps, hipStream_t s);

// Host-side jump math (same tables the device uses).
void host_jump_pow2(uint32_t state[6], uint64_t k, bool stream_tables);  // A^(k [*2^127]) state

}  // namespace mrg355
