// Storage policies for the shifted populations g_i = f_i - w_i rho0.
//
// Each policy fixes the element type in HBM, the arithmetic type of the sweep
// and the porosity-control element type:
//   StoreF64   : f64 in HBM, f64 arithmetic, d in f64   (validation form)
//   StoreF32   : f32 in HBM, f32 arithmetic, d in f32
//   StoreF16S  : f16 holding s*g (s a power of two), f32 arithmetic, d in f16
//   StoreBF16S : bf16 holding s*g, f32 arithmetic, d in f16
// Stores round to nearest even; scaling by a power of two is exact, so the
// only rounding on the way in and out is the 16-bit conversion.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hlbm {

struct StoreF64 {
    using T = double;
    using R = double;  // arithmetic type
    using D = double;  // porosity element
    static constexpr int code = 0;
    static constexpr bool exact_moments = true;  // FP64 moment sums + balance-law correction
    __device__ static inline R load(T v, R) { return v; }
    __device__ static inline T store(R v, R) { return v; }
    __device__ static inline R load_d(D v) { return v; }
};

struct StoreF32 {
    using T = float;
    using R = float;
    using D = float;
    static constexpr int code = 1;
    static constexpr bool exact_moments = true;
    __device__ static inline R load(T v, R) { return v; }
    __device__ static inline T store(R v, R) { return v; }
    __device__ static inline R load_d(D v) { return v; }
};

struct StoreF16S {
    using T = _Float16;
    using R = float;
    using D = _Float16;
    static constexpr int code = 2;
    static constexpr bool exact_moments = false;  // moment sums in f32
    __device__ static inline R load(T v, R inv_scale) { return static_cast<float>(v) * inv_scale; }
    // f32 -> f16 conversion rounds to nearest even in the default mode.
    __device__ static inline T store(R v, R scale) { return static_cast<_Float16>(v * scale); }
    __device__ static inline R load_d(D v) { return static_cast<float>(v); }
};

// bfloat16 kept as raw 16-bit patterns.  Widening is exact (the pattern is the
// upper half of an f32); narrowing rounds to nearest even by adding
// 0x7fff + lsb to the f32 pattern before truncation (values here are finite).
struct StoreBF16S {
    using T = uint16_t;
    using R = float;
    using D = _Float16;
    static constexpr int code = 3;
    static constexpr bool exact_moments = false;
    __device__ static inline R load(T v, R inv_scale)
    {
        return __uint_as_float(static_cast<uint32_t>(v) << 16) * inv_scale;
    }
    __device__ static inline T store(R v, R scale)
    {
        uint32_t u = __float_as_uint(v * scale);
        u += 0x7fffu + ((u >> 16) & 1u);
        return static_cast<uint16_t>(u >> 16);
    }
    __device__ static inline R load_d(D v) { return static_cast<float>(v); }
};

}  // namespace hlbm
