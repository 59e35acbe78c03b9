// mrg_tuned.h -- launch shapes of mrg_generate's automatic plan, per output
// kind and size class.  Results never depend on them: every value is a
// function of (stream, draw index) only.
//
// Written by `python -m paper_2201_06604_amd.tune_plain --write` from timings
// on MI355X (the tuner times candidate shapes on a representative workload of
// each class and keeps the fastest; its docstring lists them).
#pragma once

#include <stdint.h>

namespace mrg355 {

struct TunedShape {
    uint16_t spl;        // streams per lane asked for (then narrowed to what the shape allows)
    uint16_t block;      // threads per block
    uint16_t waves;      // waves the grid aims at (sets the chunk)
    uint16_t min_units;  // shortest chunk, draw units
    uint16_t lock;       // 1 = lockstep rows once the grid has two waves per SIMD
    uint16_t xcd;        // 1 = XCD-contiguous block order
};

// Kinds: uniform f64, uniform f32, raw u32, normal f64, normal f32,
// exponential f64, exponential f32.  Size classes by the call's draw count n:
// below 2^18, 2^22, 2^26, 2^29, and above (timed at 2^16, 2^20, 2^24, 2^28
// and 2^30 draws: 256 x 256, 1,024 x 1,024, 16,384 x 1,024, 65,536 x 4,096
// and 262,144 x 4,096 streams x draws).
constexpr int kTunedKinds = 7;
constexpr int kTunedClasses = 5;
// Timings of the tuning run that wrote this table (MI355X, median of 7 launches):
// uniform f64, 256 x 256: 19.4 us (entry before: 20.4 us; 12 shapes timed)
// uniform f32, 256 x 256: 19.2 us (entry before: 19.2 us; 12 shapes timed)
// raw u32, 256 x 256: 18.9 us (entry before: 19.7 us; 12 shapes timed)
// normal f64, 256 x 256: 25.4 us (entry before: 25.4 us; 8 shapes timed)
// normal f32, 256 x 256: 23.6 us (entry before: 25.0 us; 8 shapes timed)
// exponential f64, 256 x 256: 21.8 us (entry before: 21.8 us; 12 shapes timed)
// exponential f32, 256 x 256: 21.2 us (entry before: 22.4 us; 12 shapes timed)
// uniform f64, 1024 x 1024: 19.4 us (entry before: 20.0 us; 12 shapes timed)
// uniform f32, 1024 x 1024: 19.3 us (entry before: 19.9 us; 12 shapes timed)
// raw u32, 1024 x 1024: 19.5 us (entry before: 19.5 us; 12 shapes timed)
// normal f64, 1024 x 1024: 26.2 us (entry before: 26.2 us; 13 shapes timed)
// normal f32, 1024 x 1024: 25.0 us (entry before: 25.0 us; 13 shapes timed)
// exponential f64, 1024 x 1024: 22.5 us (entry before: 22.5 us; 12 shapes timed)
// exponential f32, 1024 x 1024: 22.0 us (entry before: 22.0 us; 12 shapes timed)
// uniform f64, 16384 x 1024: 36.4 us (entry before: 38.4 us; 60 shapes timed)
// uniform f32, 16384 x 1024: 28.5 us (entry before: 30.6 us; 32 shapes timed)
// raw u32, 16384 x 1024: 28.8 us (entry before: 31.3 us; 32 shapes timed)
// normal f64, 16384 x 1024: 46.6 us (entry before: 47.7 us; 28 shapes timed)
// normal f32, 16384 x 1024: 41.6 us (entry before: 43.5 us; 28 shapes timed)
// exponential f64, 16384 x 1024: 43.7 us (entry before: 50.1 us; 36 shapes timed)
// exponential f32, 16384 x 1024: 38.6 us (entry before: 41.7 us; 36 shapes timed)
// uniform f64, 65536 x 4096: 359.4 us (entry before: 368.6 us; 72 shapes timed)
// uniform f32, 65536 x 4096: 197.9 us (entry before: 197.9 us; 44 shapes timed)
// raw u32, 65536 x 4096: 183.1 us (entry before: 183.1 us; 44 shapes timed)
// normal f64, 65536 x 4096: 451.8 us (entry before: 465.2 us; 44 shapes timed)
// normal f32, 65536 x 4096: 353.9 us (entry before: 370.0 us; 44 shapes timed)
// exponential f64, 65536 x 4096: 398.3 us (entry before: 431.4 us; 40 shapes timed)
// exponential f32, 65536 x 4096: 311.1 us (entry before: 345.3 us; 40 shapes timed)
// uniform f64, 262144 x 4096: 1364.7 us (entry before: 1364.7 us; 56 shapes timed)
// uniform f32, 262144 x 4096: 763.0 us (entry before: 792.1 us; 32 shapes timed)
// raw u32, 262144 x 4096: 758.7 us (entry before: 758.7 us; 32 shapes timed)
// normal f64, 262144 x 4096: 1802.9 us (entry before: 1841.1 us; 28 shapes timed)
// normal f32, 262144 x 4096: 1364.1 us (entry before: 1424.4 us; 28 shapes timed)
// exponential f64, 262144 x 4096: 1565.9 us (entry before: 1652.8 us; 28 shapes timed)
// exponential f32, 262144 x 4096: 1192.4 us (entry before: 1241.9 us; 28 shapes timed)
// clang-format off
constexpr TunedShape kTuned[kTunedKinds][kTunedClasses] = {
    {{1, 512, 1024, 32, 0, 0}, {1, 256, 1024, 32, 0, 1}, {1, 256, 8192, 32, 1, 0}, {1, 256, 1024, 32, 0, 0}, {2, 512, 2048, 96, 1, 1}},  // uniform f64
    {{1, 256, 1024, 32, 0, 1}, {1, 256, 1024, 32, 0, 0}, {1, 256, 2048, 32, 0, 0}, {1, 256, 16384, 32, 0, 0}, {4, 256, 8192, 32, 0, 0}},  // uniform f32
    {{1, 512, 1024, 32, 0, 0}, {1, 256, 1024, 32, 0, 0}, {1, 256, 4096, 32, 0, 0}, {1, 256, 8192, 32, 0, 0}, {4, 256, 8192, 32, 0, 0}},  // raw u32
    {{1, 256, 8192, 32, 0, 1}, {1, 256, 8192, 32, 0, 1}, {2, 256, 2048, 32, 0, 1}, {2, 256, 8192, 32, 0, 0}, {2, 512, 16384, 32, 0, 0}},  // normal f64
    {{1, 256, 1024, 32, 0, 0}, {1, 256, 8192, 32, 0, 1}, {2, 256, 2048, 32, 0, 0}, {2, 256, 4096, 32, 0, 0}, {2, 512, 16384, 32, 0, 1}},  // normal f32
    {{1, 256, 4096, 32, 0, 1}, {1, 256, 4096, 32, 0, 1}, {1, 256, 2048, 32, 0, 1}, {1, 256, 8192, 32, 0, 0}, {2, 512, 16384, 32, 0, 0}},  // exponential f64
    {{1, 256, 1024, 32, 0, 0}, {1, 256, 4096, 32, 0, 1}, {2, 256, 2048, 32, 0, 0}, {2, 512, 8192, 32, 0, 0}, {2, 512, 8192, 32, 0, 1}},  // exponential f32
};
// clang-format on

}  // namespace mrg355
