// Matrix-core helpers and the LDS plane layout shared by the Theta kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace wig2 {
namespace mf {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

template <typename T>
struct Acc;
template <>
struct Acc<double> {
    typedef d4 V;
};
template <>
struct Acc<float> {
    typedef f4 V;
};

__device__ inline d4 mma(double a, double b, d4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ inline f4 mma(float a, float b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// Output-tile row held in accumulator element q of lane group lk (l / 16):
// the f32 16x16x4 instruction packs rows 4*lk + q, the f64 one rows 4*q + lk.
template <typename T>
__device__ inline int acc_row(int lk, int q);
template <>
__device__ inline int acc_row<double>(int lk, int q)
{
    return 4 * q + lk;
}
template <>
__device__ inline int acc_row<float>(int lk, int q)
{
    return 4 * lk + q;
}

template <typename T>
__device__ inline T sgnval(int d, T v)
{
    return d > 0 ? v : (d < 0 ? -v : T(0));
}

// LDS plane layout: rows of NK values at pitch LD = NK + kPadCols with
// kPadFront zero elements before row 0 and kPadCols after the last row.  The
// zero gaps make every skewed read X[k][s - k] of a tile that meets the valid
// band land on data or on a zero, so the pair-term operand needs no bounds
// test (its column stays within [-18, NK + 17]).
constexpr int kPadCols = 20;
constexpr int kPadFront = 24;

// Bytes of one padded plane plus the three signed Toeplitz tables.
template <typename T, int NK>
struct Plane {
    static constexpr int LD = NK + kPadCols;
    static constexpr int X_ELEMS = kPadFront + NK * LD + kPadCols;
    static constexpr int TAB = 2 * NK;  // signed Toeplitz tables, index d + NK
    static constexpr size_t bytes = sizeof(T) * (size_t)(X_ELEMS + 3 * TAB);
};

}  // namespace mf
}  // namespace wig2
