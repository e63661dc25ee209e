// Theta application: the pseudo-differential operator of the two-body Wigner
// equation, one x-pair momentum plane per workgroup, on gfx950 matrix cores.
//
// For the plane F = f(x_i1, x_i2, ., .) (nk x nk, n2 fastest):
//   Theta F = K1 F + F K2^T + Theta_12(F)
//   K1[r][k] = sgn(r-k) s1[|r-k|]      (Sec. 3.1.1, single-body symbol of x_i1)
//   K2[c][k] = sgn(c-k) s2[|c-k|]      (same for particle 2, x_i2)
//   Theta_12(n1,n2) = sum_m kap(m) F(n1-m, n2+m),  kap(-m) = -kap(m)
//                                      (Sec. 3.1.2, eq. two_body_FSM)
// with f = 0 outside the p-box.  On a box (Sec. 3.2.1) K1, K2 are the dense
// SEM matrices of x_i1, x_i2 and there is no pair term.
//
// The pair term runs along anti-diagonals s = n1 + n2.  In skewed coordinates
// H[n1'][s] = F[n1'][s - n1'] it is the product T H with the Toeplitz matrix
// T[n1][n1'] = kap(n1 - n1'), evaluated on 16x16 output tiles in (n1, s) that
// meet the valid parallelogram 0 <= s - n1 < nk, contracting only over the
// n1' blocks where H is non-zero.  Its tiles are scattered back into the LDS
// plane after all waves have read it, then added to the regular tiles.
//
// Work split: wave w owns output rows [16w, 16w+16) (nk/16 waves).  Operands:
// the plane in LDS (one HBM read per plane), Toeplitz operands generated from
// the symbol rows held in LDS, SEM matrices streamed from L2.
//
// Numerics: FP64 path on v_mfma_f64_16x16x4f64, FP32 path on
// v_mfma_f32_16x16x4f32, BF16X2 path on v_mfma_f32_16x16x32_bf16 with both
// operands split x = hi + lo (hi = RNE_bf16(x), lo = RNE_bf16(x - hi)) and
// hi*hi + hi*lo + lo*hi accumulated in FP32.  When the single-body symbols
// vanish beyond `band` modes (e.g. a few-mode V_ext), the single-body
// products only visit the k blocks within that band of each output tile.
#include "common.h"

#include <algorithm>

namespace wig2 {
namespace {

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

template <typename T>
__device__ inline T sgnval(int d, T v)
{
    return d > 0 ? v : (d < 0 ? -v : T(0));
}

// LDS row pitch (elements): one extra element per row spreads consecutive
// rows over different banks.
template <int NK>
struct Pitch {
    static constexpr int value = NK + 1;
};

// ---------------------------------------------------------------------------
// FP64 / FP32 kernel
// ---------------------------------------------------------------------------
template <typename T, int NK, bool TWO, bool SEM, int MODE>
__global__ __launch_bounds__(NK / 16 * 64) void k_theta(
    const T* u, const T* __restrict__ vin, T* out, int nx, const double* __restrict__ sig1,
    const double* __restrict__ sig2, int band, const double* __restrict__ kap,
    const double* __restrict__ ksem, double tau)
{
    typedef typename Acc<T>::V V;
    constexpr int NW = NK / 16;  // waves = row blocks
    constexpr int LD = Pitch<NK>::value;
    constexpr int NT = NW * 64;
    constexpr int NS = NW + 1;  // skewed tiles per row block

    extern __shared__ unsigned char smem_raw[];
    T* X = reinterpret_cast<T*>(smem_raw);  // [NK][LD]
    T* s1 = X + NK * LD;                    // [NK]
    T* s2 = s1 + NK;                        // [NK]
    T* kp = s2 + NK;                        // [NK]

    const long pl = blockIdx.x;
    const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
    const int ell = (i1 - i2 + nx) % nx;
    const int tid = threadIdx.x;
    const long pbase = pl * (long)NK * NK;

    for (int m = tid; m < NK; m += NT) {
        s1[m] = SEM ? T(0) : T(sig1[(long)i1 * NK + m]);
        s2[m] = SEM ? T(0) : T(sig2[(long)i2 * NK + m]);
        kp[m] = TWO ? T(kap[(long)ell * NK + m]) : T(0);
    }
    for (int idx = tid; idx < NK * NK; idx += NT) {
        T x = u[pbase + idx];
        if (MODE == 1) x += T(tau) * vin[pbase + idx];
        X[(idx / NK) * LD + (idx % NK)] = x;
    }
    __syncthreads();

    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r = 16 * w + li;  // A-operand row of this lane

    const int row0 = 16 * w + 4 * lk;  // first output row of this lane
    V acc[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[j] = V{0, 0, 0, 0};

    if constexpr (SEM) {
        const double* K1 = ksem + (long)i1 * NK * NK;
        const double* K2 = ksem + (long)i2 * NK * NK;
#pragma unroll 1
        for (int kb = 0; kb < NK / 4; ++kb) {
            const int k = 4 * kb + lk;
            const T a1 = T(K1[(long)r * NK + k]);
            const T a2 = X[r * LD + k];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) {
                const int c = 16 * cb + li;
                acc[cb] = mma(a1, X[k * LD + c], acc[cb]);
                acc[cb] = mma(a2, T(K2[(long)c * NK + k]), acc[cb]);
            }
        }
    } else {
        // K1 F: K1[r][k] vanishes for |r - k| > band, so only the k blocks
        // within band of this wave's rows contribute.
        const int kb1_lo = max(0, 16 * w - band) / 4;
        const int kb1_hi = min(NK - 1, 16 * w + 15 + band) / 4;
#pragma unroll 1
        for (int kb = kb1_lo; kb <= kb1_hi; ++kb) {
            const int k = 4 * kb + lk;
            const T a1 = sgnval(r - k, s1[abs(r - k)]);
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) acc[cb] = mma(a1, X[k * LD + 16 * cb + li], acc[cb]);
        }
        // F K2^T: K2[c][k] vanishes for |c - k| > band.
#pragma unroll 1
        for (int kb = 0; kb < NK / 4; ++kb) {
            const int k = 4 * kb + lk;
            const T a2 = X[r * LD + k];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) {
                if (4 * kb + 3 < 16 * cb - band || 4 * kb > 16 * cb + 15 + band) continue;
                const int c = 16 * cb + li;
                acc[cb] = mma(a2, sgnval(c - k, s2[abs(c - k)]), acc[cb]);
            }
        }
    }

    V sacc[NS];
    if constexpr (TWO) {
#pragma unroll
        for (int j = 0; j < NS; ++j) sacc[j] = V{0, 0, 0, 0};
        // skewed tile j covers s in [16(w+j), 16(w+j)+16); H[n1'][s] != 0
        // needs n1' in [s - NK + 1, s], i.e. blocks kb with
        // 4kb+3 >= 16(w+j) - NK + 1 and 4kb <= 16(w+j) + 15.
        const int kb_lo = max(0, (16 * w - NK + 1) / 4);
        const int kb_hi = min(NK / 4 - 1, (16 * (w + NW) + 15) / 4);
#pragma unroll 1
        for (int kb = kb_lo; kb <= kb_hi; ++kb) {
            const int k = 4 * kb + lk;
            const T a = sgnval(r - k, kp[abs(r - k)]);
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const int s0 = 16 * (w + j);
                if (4 * kb + 3 < s0 - NK + 1 || 4 * kb > s0 + 15) continue;  // wave-uniform
                const int col = s0 + li - k;
                const T b = (col >= 0 && col < NK) ? X[k * LD + col] : T(0);
                sacc[j] = mma(a, b, sacc[j]);
            }
        }
    }

    __syncthreads();  // every wave is done reading the plane

    if constexpr (TWO) {
        // scatter skewed tiles into the plane buffer: (n1, s) -> (n1, s - n1)
#pragma unroll
        for (int j = 0; j < NS; ++j) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n1 = row0 + q;
                const int n2 = 16 * (w + j) + li - n1;
                if (n2 >= 0 && n2 < NK) X[n1 * LD + n2] = sacc[j][q];
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int cb = 0; cb < NW; ++cb) {
        const int c = 16 * cb + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rr = row0 + q;
            T val = acc[cb][q];
            if constexpr (TWO) val += X[rr * LD + c];
            const long gi = pbase + (long)rr * NK + c;
            if (MODE == 0)
                out[gi] = val;
            else
                out[gi] = u[gi] + T(0.5 * tau) * (vin[gi] + val);
        }
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 kernel (FP32 state).  Operands are split into hi + lo bf16 and
// contracted on v_mfma_f32_16x16x32_bf16 (K = 32 per instruction): lane l
// supplies A[l%16][8(l/16) .. 8(l/16)+7] and B[8(l/16) .. +7][l%16].
// ---------------------------------------------------------------------------
__device__ inline short bf16_bits(float x)
{
    // round to nearest even
    unsigned u = __float_as_uint(x);
    unsigned r = u + 0x7FFFu + ((u >> 16) & 1u);
    return (short)(r >> 16);
}
__device__ inline float bf16_val(short b)
{
    return __uint_as_float(((unsigned)(unsigned short)b) << 16);
}

__device__ inline f4 mma_bf16(s8 a, s8 b, f4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

template <int NK, bool TWO, int MODE>
__global__ __launch_bounds__(NK / 16 * 64) void k_theta_bf16(
    const float* u, const float* __restrict__ vin, float* out, int nx,
    const double* __restrict__ sig1, const double* __restrict__ sig2, int band,
    const double* __restrict__ kap, double tau)
{
    constexpr int NW = NK / 16;
    constexpr int LD = NK + 1;
    constexpr int NT = NW * 64;
    constexpr int NS = NW + 1;
    extern __shared__ unsigned char smem_raw[];
    float* X = reinterpret_cast<float*>(smem_raw);
    float* s1 = X + NK * LD;
    float* s2 = s1 + NK;
    float* kp = s2 + NK;

    const long pl = blockIdx.x;
    const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
    const int ell = (i1 - i2 + nx) % nx;
    const int tid = threadIdx.x;
    const long pbase = pl * (long)NK * NK;
    for (int m = tid; m < NK; m += NT) {
        s1[m] = (float)sig1[(long)i1 * NK + m];
        s2[m] = (float)sig2[(long)i2 * NK + m];
        kp[m] = TWO ? (float)kap[(long)ell * NK + m] : 0.f;
    }
    for (int idx = tid; idx < NK * NK; idx += NT) {
        float x = u[pbase + idx];
        if (MODE == 1) x += (float)tau * vin[pbase + idx];
        X[(idx / NK) * LD + (idx % NK)] = x;
    }
    __syncthreads();

    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r = 16 * w + li;
    const int row0 = 16 * w + 4 * lk;
    f4 acc[NW];
#pragma unroll
    for (int j = 0; j < NW; ++j) acc[j] = f4{0, 0, 0, 0};

    auto split = [](float x, short& h, short& l) {
        h = bf16_bits(x);
        l = bf16_bits(x - bf16_val(h));
    };

    {
        // K1 F over the 32-wide k chunks within band of this wave's rows
        const int kc1_lo = max(0, 16 * w - band) / 32;
        const int kc1_hi = min(NK - 1, 16 * w + 15 + band) / 32;
#pragma unroll 1
        for (int kc = kc1_lo; kc <= kc1_hi; ++kc) {
            s8 ah, al;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 32 * kc + 8 * lk + e;
                short h, l;
                split(sgnval(r - k, s1[abs(r - k)]), h, l);
                ah[e] = h;
                al[e] = l;
            }
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) {
                const int c = 16 * cb + li;
                s8 bh, bl;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    short h, l;
                    split(X[(32 * kc + 8 * lk + e) * LD + c], h, l);
                    bh[e] = h;
                    bl[e] = l;
                }
                acc[cb] = mma_bf16(ah, bh, acc[cb]);
                acc[cb] = mma_bf16(ah, bl, acc[cb]);
                acc[cb] = mma_bf16(al, bh, acc[cb]);
            }
        }
        // F K2^T
#pragma unroll 1
        for (int kc = 0; kc < NK / 32; ++kc) {
            s8 ah, al;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                short h, l;
                split(X[r * LD + 32 * kc + 8 * lk + e], h, l);
                ah[e] = h;
                al[e] = l;
            }
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) {
                if (32 * kc + 31 < 16 * cb - band || 32 * kc > 16 * cb + 15 + band) continue;
                const int c = 16 * cb + li;
                s8 bh, bl;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = 32 * kc + 8 * lk + e;
                    short h, l;
                    split(sgnval(c - k, s2[abs(c - k)]), h, l);
                    bh[e] = h;
                    bl[e] = l;
                }
                acc[cb] = mma_bf16(ah, bh, acc[cb]);
                acc[cb] = mma_bf16(ah, bl, acc[cb]);
                acc[cb] = mma_bf16(al, bh, acc[cb]);
            }
        }
    }

    f4 sacc[NS];
    if constexpr (TWO) {
#pragma unroll
        for (int j = 0; j < NS; ++j) sacc[j] = f4{0, 0, 0, 0};
#pragma unroll 1
        for (int kc = 0; kc < NK / 32; ++kc) {
            s8 ah, al;
#pragma unroll
            for (int e = 0; e < 8; ++e) {
                const int k = 32 * kc + 8 * lk + e;
                short h, l;
                split(sgnval(r - k, kp[abs(r - k)]), h, l);
                ah[e] = h;
                al[e] = l;
            }
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const int s0 = 16 * (w + j);
                if (32 * kc + 31 < s0 - NK + 1 || 32 * kc > s0 + 15) continue;
                s8 bh, bl;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const int k = 32 * kc + 8 * lk + e;
                    const int col = s0 + li - k;
                    const float b = (col >= 0 && col < NK) ? X[k * LD + col] : 0.f;
                    short h, l;
                    split(b, h, l);
                    bh[e] = h;
                    bl[e] = l;
                }
                sacc[j] = mma_bf16(ah, bh, sacc[j]);
                sacc[j] = mma_bf16(ah, bl, sacc[j]);
                sacc[j] = mma_bf16(al, bh, sacc[j]);
            }
        }
    }
    __syncthreads();

    if constexpr (TWO) {
#pragma unroll
        for (int j = 0; j < NS; ++j) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n1 = row0 + q;
                const int n2 = 16 * (w + j) + li - n1;
                if (n2 >= 0 && n2 < NK) X[n1 * LD + n2] = sacc[j][q];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int cb = 0; cb < NW; ++cb) {
        const int c = 16 * cb + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rr = row0 + q;
            float val = acc[cb][q];
            if constexpr (TWO) val += X[rr * LD + c];
            const long gi = pbase + (long)rr * NK + c;
            if (MODE == 0)
                out[gi] = val;
            else
                out[gi] = u[gi] + (float)(0.5 * tau) * (vin[gi] + val);
        }
    }
}

template <typename T, int NK>
size_t smem_bytes()
{
    return sizeof(T) * ((size_t)NK * Pitch<NK>::value + 3 * NK);
}

template <typename T, int NK, bool TWO, bool SEM>
hipError_t go(const ThetaArgs& a, const T* u, const T* v, T* out, int mode, double tau,
              hipStream_t st)
{
    const unsigned np = (unsigned)((long)a.nx * a.nx);
    const size_t sm = smem_bytes<T, NK>();
    const int band = std::min(a.band, NK - 1);
    if (mode == 0) {
        auto kf = k_theta<T, NK, TWO, SEM, 0>;
        hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        hipLaunchKernelGGL(kf, dim3(np), dim3(NK / 16 * 64), sm, st, u, v, out, a.nx, a.sig1,
                           a.sig2, band, a.kap, a.ksem, tau);
    } else {
        auto kf = k_theta<T, NK, TWO, SEM, 1>;
        hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        hipLaunchKernelGGL(kf, dim3(np), dim3(NK / 16 * 64), sm, st, u, v, out, a.nx, a.sig1,
                           a.sig2, band, a.kap, a.ksem, tau);
    }
    return hipGetLastError();
}

template <int NK, bool TWO>
hipError_t go_bf16(const ThetaArgs& a, const float* u, const float* v, float* out, int mode,
                   double tau, hipStream_t st)
{
    const unsigned np = (unsigned)((long)a.nx * a.nx);
    const size_t sm = smem_bytes<float, NK>();
    const int band = std::min(a.band, NK - 1);
    if (mode == 0) {
        auto kf = k_theta_bf16<NK, TWO, 0>;
        hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        hipLaunchKernelGGL(kf, dim3(np), dim3(NK / 16 * 64), sm, st, u, v, out, a.nx, a.sig1,
                           a.sig2, band, a.kap, tau);
    } else {
        auto kf = k_theta_bf16<NK, TWO, 1>;
        hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        hipLaunchKernelGGL(kf, dim3(np), dim3(NK / 16 * 64), sm, st, u, v, out, a.nx, a.sig1,
                           a.sig2, band, a.kap, tau);
    }
    return hipGetLastError();
}

template <typename T, int NK>
hipError_t dispatch_nk(const ThetaArgs& a, const T* u, const T* v, T* out, int mode, double tau,
                       hipStream_t st)
{
    const bool two = a.kap != nullptr;
    if (a.ksem) {
        if (two) return hipErrorNotSupported;
        return go<T, NK, false, true>(a, u, v, out, mode, tau, st);
    }
    if constexpr (sizeof(T) == 4) {
        if (a.precision == WIG2_BF16X2) {
            if constexpr (NK % 32 == 0) {
                const float* uf = reinterpret_cast<const float*>(u);
                const float* vf = reinterpret_cast<const float*>(v);
                float* of = reinterpret_cast<float*>(out);
                return two ? go_bf16<NK, true>(a, uf, vf, of, mode, tau, st)
                           : go_bf16<NK, false>(a, uf, vf, of, mode, tau, st);
            } else {
                return hipErrorNotSupported;
            }
        }
    }
    return two ? go<T, NK, true, false>(a, u, v, out, mode, tau, st)
               : go<T, NK, false, false>(a, u, v, out, mode, tau, st);
}

}  // namespace

template <typename T>
hipError_t launch_theta(const ThetaArgs& a, const T* u, const T* v, T* out, int mode, double tau,
                        hipStream_t st)
{
    switch (a.nk) {
    case 16: return dispatch_nk<T, 16>(a, u, v, out, mode, tau, st);
    case 32: return dispatch_nk<T, 32>(a, u, v, out, mode, tau, st);
    case 48: return dispatch_nk<T, 48>(a, u, v, out, mode, tau, st);
    case 64: return dispatch_nk<T, 64>(a, u, v, out, mode, tau, st);
    case 96: return dispatch_nk<T, 96>(a, u, v, out, mode, tau, st);
    case 128: return dispatch_nk<T, 128>(a, u, v, out, mode, tau, st);
    default: return hipErrorNotSupported;
    }
}

template hipError_t launch_theta<double>(const ThetaArgs&, const double*, const double*, double*,
                                         int, double, hipStream_t);
template hipError_t launch_theta<float>(const ThetaArgs&, const float*, const float*, float*, int,
                                        double, hipStream_t);

}  // namespace wig2
