// Learned surrogate for the pair-interaction increment over a block of fine
// steps (the Theta[V12] part of the two-body operator, Sec. 3.1.2): a small
// per-point MLP
//   y(x) = w3 . tanh(W2 tanh(W1 x + b1) + b2) + b3 + a . x,
// reads the block-start state along the anti-diagonal through the point (the
// direction the pair term couples, l = i1 - i2) and predicts the increment
// Delta / s_out.  Its inputs follow the form of the pair term, whose kernel
// is V12_m sin(2 pi m l / nx) on the antisymmetric differences
// d_m = f(n1 - m, n2 + m) - f(n1 + m, n2 - m) (its square brings in
// cos(2 pi m l / nx) on the symmetric sums e_m = f(n1 - m, n2 + m) +
// f(n1 + m, n2 - m)):
//   x = [s_in f_t(n1, n2);  s_in sin(2 pi m l/nx) d_m, m = 1..R;
//        s_in cos(2 pi m l/nx) e_m, m = 1..R;  sin(2 pi l/nx), cos(2 pi l/nx), U]
// with f_t = 0 off the p-box.  Training: minibatch MSE with Adam; per workgroup the
// forward and backward passes of 256 sample points run in registers, the
// per-sample activations go to LDS and the weight gradients are their sums
// over the 256 samples (one partial per workgroup, reduced in the update
// kernel).  Inference uses the BF16-rounded weights with FP32 arithmetic.
#include "common.h"

#include <cmath>

namespace wig2 {
namespace {

constexpr int R = kSurR, H = kSurH, D = kSurD, P = kSurP;
constexpr int OW1 = 0, OB1 = H * D, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H, OB3 = OW3 + H;
constexpr int OA = OB3 + 1;  // linear path a[D]
static_assert(OA + D == P, "parameter layout");
constexpr int TB = 256;  // samples per workgroup

struct PointIdx {
    long pl;
    int n1, n2;
    float cs, cc;
};

__device__ inline PointIdx decode(long idx, int nx, int nk)
{
    PointIdx q;
    q.n2 = (int)(idx % nk);
    q.n1 = (int)((idx / nk) % nk);
    q.pl = idx / ((long)nk * nk);
    const int i1 = (int)(q.pl / nx), i2 = (int)(q.pl % nx);
    const int ell = (i1 - i2 + nx) % nx;
    const float ang = 6.283185307179586f * (float)ell / (float)nx;
    q.cs = sinf(ang);
    q.cc = cosf(ang);
    return q;
}

template <typename T>
__device__ inline void features(const T* ft, const PointIdx& q, int nk, const SurScales& sc, float x[D])
{
    const T* F = ft + q.pl * (long)nk * nk;
    auto at = [&](int m) {  // s_in f_t(n1 - m, n2 + m), zero off the p-box
        const int a = q.n1 - m, b = q.n2 + m;
        return (a >= 0 && a < nk && b >= 0 && b < nk) ? sc.in_scale * (float)F[(long)a * nk + b] : 0.f;
    };
    x[0] = at(0);
    // sin / cos of m * 2 pi l / nx by the angle-addition recurrence
    float sm = q.cs, cm = q.cc;
#pragma unroll
    for (int m = 1; m <= R; ++m) {
        const float lo = at(m), hi = at(-m);
        x[m] = sm * (lo - hi);
        x[R + m] = cm * (lo + hi);
        const float sn = sm * q.cc + cm * q.cs;
        cm = cm * q.cc - sm * q.cs;
        sm = sn;
    }
    x[2 * R + 1] = q.cs;
    x[2 * R + 2] = q.cc;
    x[2 * R + 3] = sc.u_feat;
}

__device__ inline float forward(const float* W, const float x[D], float h1[H], float h2[H])
{
#pragma unroll
    for (int h = 0; h < H; ++h) {
        float z = W[OB1 + h];
#pragma unroll
        for (int d = 0; d < D; ++d) z += W[OW1 + h * D + d] * x[d];
        h1[h] = tanhf(z);
    }
#pragma unroll
    for (int h = 0; h < H; ++h) {
        float z = W[OB2 + h];
#pragma unroll
        for (int j = 0; j < H; ++j) z += W[OW2 + h * H + j] * h1[j];
        h2[h] = tanhf(z);
    }
    float y = W[OB3];
#pragma unroll
    for (int h = 0; h < H; ++h) y += W[OW3 + h] * h2[h];
#pragma unroll
    for (int d = 0; d < D; ++d) y += W[OA + d] * x[d];
    return y;
}

__device__ inline float block_sum(float v, float* red)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) red[w] = v;
    __syncthreads();
    float s = 0.f;
    if (threadIdx.x == 0)
        for (int i = 0; i < TB / 64; ++i) s += red[i];
    return s;  // valid in thread 0
}

// One workgroup: 256 samples idx = (p0 + k) * mul + off mod npts, k < count.
// TRAIN: writes the 625 gradient sums (of (y - t) dy/dW) to partial[block];
// always writes the sum of (y - t)^2 to lpart[block].
template <typename T, bool TRAIN>
__global__ __launch_bounds__(TB) void k_sur_batch(const T* ft, const T* delta, int nx, int nk, long npts,
                                                  long k0, long count, long mul, long off, SurScales sc,
                                                  const float* __restrict__ params, float* partial,
                                                  float* lpart)
{
    __shared__ float W[P];
    __shared__ float X[TB][D + 1];
    __shared__ float DZ1[TB][H + 1];
    __shared__ float H1[TB][H + 1];
    __shared__ float DZ2[TB][H + 1];
    __shared__ float H2[TB][H + 1];
    __shared__ float DY[TB];
    __shared__ float red[TB / 64];
    const int tid = threadIdx.x;
    for (int j = tid; j < P; j += TB) W[j] = params[j];
    __syncthreads();

    const long k = (long)blockIdx.x * TB + tid;
    float x[D], h1[H], h2[H], dy = 0.f;
    bool valid = k < count;
    if (valid) {
        const long idx = ((k0 + k) % npts * mul + off) % npts;
        const PointIdx q = decode(idx, nx, nk);
        features(ft, q, nk, sc, x);
        const float y = forward(W, x, h1, h2);
        dy = y - sc.inv_out_scale * (float)delta[idx];
    } else {
#pragma unroll
        for (int d = 0; d < D; ++d) x[d] = 0.f;
#pragma unroll
        for (int h = 0; h < H; ++h) h1[h] = h2[h] = 0.f;
    }
    const float ls = block_sum(dy * dy, red);
    if (tid == 0) lpart[blockIdx.x] = ls;
    if constexpr (TRAIN) {
        float dz2[H], dz1[H];
#pragma unroll
        for (int h = 0; h < H; ++h) dz2[h] = W[OW3 + h] * dy * (1.f - h2[h] * h2[h]);
#pragma unroll
        for (int j = 0; j < H; ++j) {
            float s = 0.f;
#pragma unroll
            for (int h = 0; h < H; ++h) s += W[OW2 + h * H + j] * dz2[h];
            dz1[j] = s * (1.f - h1[j] * h1[j]);
        }
#pragma unroll
        for (int d = 0; d < D; ++d) X[tid][d] = x[d];
#pragma unroll
        for (int h = 0; h < H; ++h) {
            DZ1[tid][h] = dz1[h];
            H1[tid][h] = h1[h];
            DZ2[tid][h] = dz2[h];
            H2[tid][h] = h2[h];
        }
        DY[tid] = dy;
        __syncthreads();
        for (int j = tid; j < P; j += TB) {
            float g = 0.f;
            if (j < OB1) {
                const int h = j / D, d = j % D;
                for (int s = 0; s < TB; ++s) g += DZ1[s][h] * X[s][d];
            } else if (j < OW2) {
                const int h = j - OB1;
                for (int s = 0; s < TB; ++s) g += DZ1[s][h];
            } else if (j < OB2) {
                const int h = (j - OW2) / H, i = (j - OW2) % H;
                for (int s = 0; s < TB; ++s) g += DZ2[s][h] * H1[s][i];
            } else if (j < OW3) {
                const int h = j - OB2;
                for (int s = 0; s < TB; ++s) g += DZ2[s][h];
            } else if (j < OB3) {
                const int h = j - OW3;
                for (int s = 0; s < TB; ++s) g += DY[s] * H2[s][h];
            } else if (j == OB3) {
                for (int s = 0; s < TB; ++s) g += DY[s];
            } else {
                const int d = j - OA;
                for (int s = 0; s < TB; ++s) g += DY[s] * X[s][d];
            }
            partial[(long)blockIdx.x * P + j] = g;
        }
    }
}

__device__ inline unsigned short to_bf16(float v)
{
    const unsigned u = __float_as_uint(v);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}

// Sum the per-workgroup gradients (scaled by gscale) and take one Adam step
// (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected); refresh the BF16 copy.
__global__ void k_sur_adam(float* params, float* mom, float* var, unsigned short* pbf,
                           const float* __restrict__ partial, int nwg, float gscale, float lr, int step,
                           float* grad_out)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= P) return;
    float g = 0.f;
    for (int w = 0; w < nwg; ++w) g += partial[(long)w * P + j];
    g *= gscale;
    if (grad_out) {
        grad_out[j] = g;
        return;
    }
    const float b1 = 0.9f, b2 = 0.999f;
    const float m = b1 * mom[j] + (1.f - b1) * g;
    const float v = b2 * var[j] + (1.f - b2) * g * g;
    mom[j] = m;
    var[j] = v;
    const float mh = m / (1.f - powf(b1, (float)step));
    const float vh = v / (1.f - powf(b2, (float)step));
    const float p = params[j] - lr * mh / (sqrtf(vh) + 1e-8f);
    params[j] = p;
    pbf[j] = to_bf16(p);
}

// Inference: f[idx] += s_out * y(features of ft at idx), BF16 weights.
template <typename T>
__global__ __launch_bounds__(TB) void k_sur_apply(const T* ft, T* f, int nx, int nk, long npts, SurScales sc,
                                                  const unsigned short* __restrict__ pbf)
{
    __shared__ float W[P];
    for (int j = threadIdx.x; j < P; j += TB) W[j] = __uint_as_float(((unsigned)pbf[j]) << 16);
    __syncthreads();
    const long idx = (long)blockIdx.x * TB + threadIdx.x;
    if (idx >= npts) return;
    const PointIdx q = decode(idx, nx, nk);
    float x[D], h1[H], h2[H];
    features(ft, q, nk, sc, x);
    const float y = forward(W, x, h1, h2);
    f[idx] = f[idx] + (T)(sc.out_scale * y);
}

// d = a - b elementwise (T), and per-workgroup max|a - b| and max|b|.
template <typename T>
__global__ __launch_bounds__(TB) void k_diff_max(const T* a, const T* b, T* d, long n, float* part)
{
    __shared__ float r1[TB / 64], r2[TB / 64];
    float m1 = 0.f, m2 = 0.f;
    for (long i = (long)blockIdx.x * TB + threadIdx.x; i < n; i += (long)gridDim.x * TB) {
        const T di = a[i] - b[i];
        if (d) d[i] = di;
        m1 = fmaxf(m1, fabsf((float)di));
        m2 = fmaxf(m2, fabsf((float)b[i]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        m1 = fmaxf(m1, __shfl_xor(m1, o));
        m2 = fmaxf(m2, __shfl_xor(m2, o));
    }
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    if (lane == 0) {
        r1[w] = m1;
        r2[w] = m2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < TB / 64; ++i) {
            m1 = fmaxf(m1, r1[i]);
            m2 = fmaxf(m2, r2[i]);
        }
        m1 = fmaxf(m1, r1[0]);
        m2 = fmaxf(m2, r2[0]);
        part[2 * blockIdx.x] = m1;
        part[2 * blockIdx.x + 1] = m2;
    }
}

}  // namespace

template <typename T>
hipError_t launch_sur_batch(const T* ft, const T* delta, int nx, int nk, long npts, long k0, long count,
                            long mul, long off, const SurScales& sc, const float* params, float* partial,
                            float* lpart, bool train, hipStream_t st)
{
    const unsigned nb = (unsigned)((count + TB - 1) / TB);
    if (train)
        hipLaunchKernelGGL((k_sur_batch<T, true>), dim3(nb), dim3(TB), 0, st, ft, delta, nx, nk, npts, k0,
                           count, mul, off, sc, params, partial, lpart);
    else
        hipLaunchKernelGGL((k_sur_batch<T, false>), dim3(nb), dim3(TB), 0, st, ft, delta, nx, nk, npts, k0,
                           count, mul, off, sc, params, partial, lpart);
    return hipGetLastError();
}

hipError_t launch_sur_adam(float* params, float* mom, float* var, unsigned short* pbf, const float* partial,
                           int nwg, float gscale, float lr, int step, float* grad_out, hipStream_t st)
{
    hipLaunchKernelGGL(k_sur_adam, dim3((P + 255) / 256), dim3(256), 0, st, params, mom, var, pbf, partial,
                       nwg, gscale, lr, step, grad_out);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sur_apply(const T* ft, T* f, int nx, int nk, const SurScales& sc, const unsigned short* pbf,
                            hipStream_t st)
{
    const long npts = (long)nx * nx * nk * nk;
    hipLaunchKernelGGL(k_sur_apply<T>, dim3((unsigned)((npts + TB - 1) / TB)), dim3(TB), 0, st, ft, f, nx,
                       nk, npts, sc, pbf);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diff_max(const T* a, const T* b, T* d, long n, float* part, int nwg, hipStream_t st)
{
    hipLaunchKernelGGL(k_diff_max<T>, dim3(nwg), dim3(TB), 0, st, a, b, d, n, part);
    return hipGetLastError();
}

template hipError_t launch_sur_batch<float>(const float*, const float*, int, int, long, long, long, long, long,
                                            const SurScales&, const float*, float*, float*, bool, hipStream_t);
template hipError_t launch_sur_batch<double>(const double*, const double*, int, int, long, long, long, long,
                                             long, const SurScales&, const float*, float*, float*, bool,
                                             hipStream_t);
template hipError_t launch_sur_apply<float>(const float*, float*, int, int, const SurScales&,
                                            const unsigned short*, hipStream_t);
template hipError_t launch_sur_apply<double>(const double*, double*, int, int, const SurScales&,
                                             const unsigned short*, hipStream_t);
template hipError_t launch_diff_max<float>(const float*, const float*, float*, long, float*, int, hipStream_t);
template hipError_t launch_diff_max<double>(const double*, const double*, double*, long, float*, int,
                                            hipStream_t);

}  // namespace wig2
