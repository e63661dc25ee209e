// Dense two-sided Theta for momentum planes larger than one CU's LDS: the
// non-periodic single-body operator of Sec. 3.2.1 (eq. Chebyshev_PDO) gives,
// per x node, a dense SEM matrix K_i, and per x-pair plane F
//   Theta F = K_{i1} F + F K_{i2}^T.
// Each workgroup computes an NK x NC block of one plane's result as a
// two-term GEMM over k panels of KP: the four operand panels (K1[:, k],
// F[:, k], F[k, cols], K2[cols, k]) pass through LDS, the next panel's
// global loads are in flight in registers while the matrix cores work on the
// current one.  Wave w owns rows [16w, 16w + 16) and all NC/16 column tiles.
//
// Workgroups are ordered so that each XCD walks a contiguous range of planes:
// consecutive planes share K_{i1}, which then stays in that XCD's L2.
//
// Precisions: FP64 on v_mfma_f64_16x16x4f64, FP32 on v_mfma_f32_16x16x4f32,
// split-BF16 (FP32 state) on v_mfma_f32_16x16x32_bf16 with both operands
// stored in LDS as hi + lo (hi = RNE_bf16(x), lo = RNE_bf16(x - hi)) and
// hi*hi + hi*lo + lo*hi accumulated in FP32.
//
// Epilogue forms as for the streaming kernel:
//   form 0: out = Theta[x];  form 1: out = x + tau Theta[x];
//   form 2: out = (y + x)/2 + (tau/2) Theta[x].
// out may alias y; out may alias x only when one workgroup covers a whole
// plane (NC == NK), which the launcher checks.
#include "common.h"
#include "mfma.h"

#include <algorithm>

namespace wig2 {
namespace {
using namespace mf;

constexpr int kPanelNk = 256;

// Per precision: RB row blocks of 16 per wave (NK / (16 RB) waves) and NC
// result columns per workgroup, sized so that accumulators and the prefetch
// registers fit the waves a SIMD holds.
template <typename T>
struct PanelShape;
template <>
struct PanelShape<double> {
    static constexpr int RB = 2;    // 8 waves, 2 x 8 tiles x 8 VGPRs of accumulators
    static constexpr int NC = 128;
    static constexpr int KP = 8;
    static constexpr int PADA = 2;
};
template <>
struct PanelShape<float> {
    static constexpr int RB = 1;    // 16 waves, 16 tiles x 4 VGPRs
    static constexpr int NC = 256;
    static constexpr int KP = 16;
    static constexpr int PADA = 4;
};

template <typename T, int NK>
struct PanelLayout {
    static constexpr int RB = PanelShape<T>::RB;
    static constexpr int NT = NK / (16 * RB) * 64;
    static constexpr int NC = PanelShape<T>::NC;
    static constexpr int KP = PanelShape<T>::KP;
    static constexpr int LDA = KP + PanelShape<T>::PADA;
    static constexpr int LDB = NC + 16;
    static constexpr size_t bytes = sizeof(T) * (size_t)(2 * NK * LDA + 2 * KP * LDB);
};

// Logical block index with each XCD (blocks are dealt round-robin over 8)
// taking one contiguous share.
__device__ inline long xcd_block(long b, long G)
{
    const long full = G / 8 * 8;
    return b < full ? (b % 8) * (G / 8) + b / 8 : b;
}

template <typename T, int NK, int FORM>
__global__ __launch_bounds__((PanelLayout<T, NK>::NT)) void k_theta_panel(const T* x, const T* y, T* out,
                                                                        int nx, const T* __restrict__ kmat,
                                                                        const T* __restrict__ kmat2, double tau)
{
    typedef typename Acc<T>::V V;
    typedef PanelLayout<T, NK> L;
    constexpr int RB = L::RB, NT = L::NT;
    constexpr int NC = L::NC, KP = L::KP, LDA = L::LDA, LDB = L::LDB;
    constexpr int NCB = NK / NC, NTILE = NC / 16, NP = NK / KP;
    constexpr int AE = NK * KP / NT;  // A-panel elements per thread
    constexpr int BE = KP * NC / NT;  // B-panel elements per thread
    static_assert(AE * NT == NK * KP && BE * NT == KP * NC, "panel split");

    extern __shared__ unsigned char smem_raw[];
    T* AK = reinterpret_cast<T*>(smem_raw);  // AK[r][kk] = K1[r][k0 + kk]
    T* AF = AK + NK * LDA;                   // AF[r][kk] = F[r][k0 + kk]
    T* BF = AF + NK * LDA;                   // BF[kk][c] = F[k0 + kk][c0 + c]
    T* BK = BF + KP * LDB;                   // BK[kk][c] = K2[c0 + c][k0 + kk]

    const long lb = xcd_block(blockIdx.x, gridDim.x);
    const long pl = lb / NCB;
    const int c0 = (int)(lb % NCB) * NC;
    const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
    const long pbase = pl * (long)NK * NK;
    const T* F = x + pbase;
    const T* K1 = kmat + (long)i1 * NK * NK;
    const T* K2 = kmat2 + (long)i2 * NK * NK;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;

    // loader coordinates
    const int ra = tid / (KP / AE), ka = (tid % (KP / AE)) * AE;    // A panels
    const int kb = tid / (NC / BE), cbf = (tid % (NC / BE)) * BE;   // F row panel
    const int ck = tid / (KP / BE), kq = (tid % (KP / BE)) * BE;    // K2 panel
    T ak[AE], af[AE], bf[BE], bk[BE];
    // per-thread operand pointers, advanced by one panel per fetch
    const T* pk1 = K1 + (long)ra * NK + ka;
    const T* pf = F + (long)ra * NK + ka;
    const T* pbf = F + (long)kb * NK + c0 + cbf;
    const T* pk2 = K2 + (long)(c0 + ck) * NK + kq;
    auto fetch = [&](int) {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            ak[e] = pk1[e];
            af[e] = pf[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            bf[e] = pbf[e];
            bk[e] = pk2[e];
        }
        pk1 += KP;
        pf += KP;
        pbf += (long)KP * NK;
        pk2 += KP;
    };
    auto stage = [&]() {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            AK[ra * LDA + ka + e] = ak[e];
            AF[ra * LDA + ka + e] = af[e];
        }
#pragma unroll
        for (int e = 0; e < BE; ++e) {
            BF[kb * LDB + cbf + e] = bf[e];
            BK[(kq + e) * LDB + ck] = bk[e];
        }
    };

    // wave w owns row blocks w*RB .. w*RB + RB - 1
    V acc[RB][NTILE];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int t = 0; t < NTILE; ++t) acc[b][t] = V{0, 0, 0, 0};

    fetch(0);
    for (int p = 0; p < NP; ++p) {
        stage();
        __syncthreads();
        if (p + 1 < NP) fetch(p + 1);
#pragma unroll
        for (int ks = 0; ks < KP / 4; ++ks) {
            const int k = 4 * ks + lk;
            T a1[RB], a2[RB];
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                a1[b] = AK[(16 * (w * RB + b) + li) * LDA + k];
                a2[b] = AF[(16 * (w * RB + b) + li) * LDA + k];
            }
#pragma unroll
            for (int t = 0; t < NTILE; ++t) {
                const T b1 = BF[k * LDB + 16 * t + li];
                const T b2 = BK[k * LDB + 16 * t + li];
#pragma unroll
                for (int b = 0; b < RB; ++b) {
                    acc[b][t] = mma(a1[b], b1, acc[b][t]);
                    acc[b][t] = mma(a2[b], b2, acc[b][t]);
                }
                if (t % 4 == 3) __builtin_amdgcn_sched_barrier(0);  // bound the reads in flight
            }
        }
        __syncthreads();
    }

#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * (w * RB + b) + acc_row<T>(lk, q);
            const long gi = pbase + (long)r * NK + c0 + 16 * t + li;
            const T val = acc[b][t][q];
            if constexpr (FORM == 0)
                out[gi] = val;
            else if constexpr (FORM == 1)
                out[gi] = x[gi] + T(tau) * val;
            else
                out[gi] = T(0.5) * (y[gi] + x[gi]) + T(0.5 * tau) * val;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

// ---------------------------------------------------------------------------
// Split-BF16 variant (FP32 state, FP32 matrices).  K panel depth 32 (one
// bf16 instruction); operands are split once when staged into LDS, A panels
// row-major [r][kk], B panels stored transposed [c][kk] so that each lane's
// 8 consecutive k are one 16-byte LDS read.
// ---------------------------------------------------------------------------
typedef float f4v __attribute__((ext_vector_type(4)));
typedef short s8v __attribute__((ext_vector_type(8)));

__device__ inline unsigned short bf16_rne(float v)
{
    const unsigned u = __float_as_uint(v);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float bf16_to_f(unsigned short b) { return __uint_as_float(((unsigned)b) << 16); }

template <int NK>
struct PanelBf16Layout {
    static constexpr int RB = 2;       // 8 waves, 2 x 8 tiles x 4 VGPRs of accumulators
    static constexpr int NT = NK / (16 * RB) * 64;
    static constexpr int NC = 128;
    static constexpr int KP = 32;
    static constexpr int LD = KP + 8;  // shorts per row: 80 bytes
    // AKh, AKl, AFh, AFl: [NK][LD]; BFh, BFl, BKh, BKl: [NC][LD]
    static constexpr size_t bytes = 2 * (size_t)(4 * NK * LD + 4 * NC * LD);
};

template <int NK, int FORM>
__global__ __launch_bounds__((PanelBf16Layout<NK>::NT)) void k_theta_panel_bf16(
    const float* x, const float* y, float* out, int nx, const float* __restrict__ kmat,
    const float* __restrict__ kmat2, double tau)
{
    typedef PanelBf16Layout<NK> L;
    constexpr int RB = L::RB, NT = L::NT;
    constexpr int NC = L::NC, KP = L::KP, LD = L::LD;
    constexpr int NCB = NK / NC, NTILE = NC / 16, NP = NK / KP;
    constexpr int AE = NK * KP / NT;  // 16: A panels, 2 chunks of 8 per thread
    constexpr int KE = NC * KP / NT;  // 8: K2 panel
    constexpr int BE = KP * NC / NT;  // 8: F row panel
    static_assert(AE == 16 && KE == 8 && BE == 8, "bf16 panel split");

    extern __shared__ unsigned char smem_raw[];
    unsigned short* S = reinterpret_cast<unsigned short*>(smem_raw);
    unsigned short* AKh = S;
    unsigned short* AKl = AKh + NK * LD;
    unsigned short* AFh = AKl + NK * LD;
    unsigned short* AFl = AFh + NK * LD;
    unsigned short* BFh = AFl + NK * LD;  // BF*[c][kk] = F[k0 + kk][c0 + c]
    unsigned short* BFl = BFh + NC * LD;
    unsigned short* BKh = BFl + NC * LD;  // BK*[c][kk] = K2[c0 + c][k0 + kk]
    unsigned short* BKl = BKh + NC * LD;

    const long lb = xcd_block(blockIdx.x, gridDim.x);
    const long pl = lb / NCB;
    const int c0 = (int)(lb % NCB) * NC;
    const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
    const long pbase = pl * (long)NK * NK;
    const float* F = x + pbase;
    const float* K1 = kmat + (long)i1 * NK * NK;
    const float* K2 = kmat2 + (long)i2 * NK * NK;

    const int tid = threadIdx.x;
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;

    // A panels: thread covers row ra, k chunk ka .. ka+15 (two 8-chunks)
    const int ra = tid / (KP / AE), ka = (tid % (KP / AE)) * AE;
    // K2 panel: row rk (result column), k chunk kk0 .. kk0+7
    const int rk = tid / (KP / KE), kk0 = (tid % (KP / KE)) * KE;
    // F row panel: k row kb, columns cbf .. cbf+7
    const int kb = tid / (NC / BE), cbf = (tid % (NC / BE)) * BE;
    float ak[AE], af[AE], bk[KE], bf[BE];
    auto fetch = [&](int p) {
        const int k0 = p * KP;
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            ak[e] = K1[(long)ra * NK + k0 + ka + e];
            af[e] = F[(long)ra * NK + k0 + ka + e];
        }
#pragma unroll
        for (int e = 0; e < KE; ++e) bk[e] = K2[(long)(c0 + rk) * NK + k0 + kk0 + e];
#pragma unroll
        for (int e = 0; e < BE; ++e) bf[e] = F[(long)(k0 + kb) * NK + c0 + cbf + e];
    };
    auto put = [&](unsigned short* hi, unsigned short* lo, int idx, float v) {
        const unsigned short h = bf16_rne(v);
        hi[idx] = h;
        lo[idx] = bf16_rne(v - bf16_to_f(h));
    };
    auto stage = [&]() {
#pragma unroll
        for (int e = 0; e < AE; ++e) {
            put(AKh, AKl, ra * LD + ka + e, ak[e]);
            put(AFh, AFl, ra * LD + ka + e, af[e]);
        }
#pragma unroll
        for (int e = 0; e < KE; ++e) put(BKh, BKl, rk * LD + kk0 + e, bk[e]);
#pragma unroll
        for (int e = 0; e < BE; ++e) put(BFh, BFl, (cbf + e) * LD + kb, bf[e]);
    };

    f4v acc[RB][NTILE];
#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
        for (int t = 0; t < NTILE; ++t) acc[b][t] = f4v{0, 0, 0, 0};

    fetch(0);
    for (int p = 0; p < NP; ++p) {
        stage();
        __syncthreads();
        if (p + 1 < NP) fetch(p + 1);
        s8v a1h[RB], a1l[RB], a2h[RB], a2l[RB];
#pragma unroll
        for (int b = 0; b < RB; ++b) {
            const int ao = (16 * (w * RB + b) + li) * LD + 8 * lk;
            a1h[b] = *reinterpret_cast<const s8v*>(AKh + ao);
            a1l[b] = *reinterpret_cast<const s8v*>(AKl + ao);
            a2h[b] = *reinterpret_cast<const s8v*>(AFh + ao);
            a2l[b] = *reinterpret_cast<const s8v*>(AFl + ao);
        }
#pragma unroll
        for (int t = 0; t < NTILE; ++t) {
            const int bo = (16 * t + li) * LD + 8 * lk;
            const s8v bfh = *reinterpret_cast<const s8v*>(BFh + bo);
            const s8v bfl = *reinterpret_cast<const s8v*>(BFl + bo);
            const s8v bkh = *reinterpret_cast<const s8v*>(BKh + bo);
            const s8v bkl = *reinterpret_cast<const s8v*>(BKl + bo);
#pragma unroll
            for (int b = 0; b < RB; ++b) {
                f4v c = acc[b][t];
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h[b], bfh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1h[b], bfl, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a1l[b], bfh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2h[b], bkh, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2h[b], bkl, c, 0, 0, 0);
                c = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a2l[b], bkh, c, 0, 0, 0);
                acc[b][t] = c;
            }
            if (t % 2 == 1) __builtin_amdgcn_sched_barrier(0);  // bound the reads in flight
        }
        __syncthreads();
    }

#pragma unroll
    for (int b = 0; b < RB; ++b)
#pragma unroll
    for (int t = 0; t < NTILE; ++t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int r = 16 * (w * RB + b) + 4 * lk + q;  // f32 accumulator rows
            const long gi = pbase + (long)r * NK + c0 + 16 * t + li;
            const float val = acc[b][t][q];
            if constexpr (FORM == 0)
                out[gi] = val;
            else if constexpr (FORM == 1)
                out[gi] = x[gi] + (float)tau * val;
            else
                out[gi] = 0.5f * (y[gi] + x[gi]) + (float)(0.5 * tau) * val;
        }
        __builtin_amdgcn_sched_barrier(0);
    }
}

template <typename T, int FORM>
hipError_t go_panel(const ThetaArgs& a, const T* x, const T* y, T* out, double tau, hipStream_t st)
{
    constexpr int NK = kPanelNk;
    const long np = (long)a.nx * a.nx;
    if constexpr (sizeof(T) == 4) {
        if (a.precision == WIG2_BF16X2) {
            auto kf = k_theta_panel_bf16<NK, FORM>;
            const size_t sm = PanelBf16Layout<NK>::bytes;
            hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
            if (e != hipSuccess) return e;
            const long nb = np * (NK / PanelBf16Layout<NK>::NC);
            hipLaunchKernelGGL(kf, dim3((unsigned)nb), dim3(PanelBf16Layout<NK>::NT), sm, st, x, y, out,
                               a.nx, reinterpret_cast<const float*>(a.ksem_t),
                               reinterpret_cast<const float*>(a.ksem2_t ? a.ksem2_t : a.ksem_t), tau);
            return hipGetLastError();
        }
    }
    auto kf = k_theta_panel<T, NK, FORM>;
    const size_t sm = PanelLayout<T, NK>::bytes;
    hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    const long nb = np * (NK / PanelLayout<T, NK>::NC);
    hipLaunchKernelGGL(kf, dim3((unsigned)nb), dim3(PanelLayout<T, NK>::NT), sm, st, x, y, out, a.nx,
                       reinterpret_cast<const T*>(a.ksem_t),
                       reinterpret_cast<const T*>(a.ksem2_t ? a.ksem2_t : a.ksem_t), tau);
    return hipGetLastError();
}

}  // namespace

bool theta_panel_ok(const ThetaArgs& a)
{
    return a.nk == kPanelNk && a.ksem_t && !a.kap;
}

template <typename T>
hipError_t launch_theta_panel(const ThetaArgs& a, const T* x, const T* y, T* out, int form, double tau,
                              hipStream_t st)
{
    if (!theta_panel_ok(a) || (form == 2 && !y)) return hipErrorNotSupported;
    // several workgroups share a plane except for FP32
    const bool whole_plane = sizeof(T) == 4 && a.precision != WIG2_BF16X2;
    if (!whole_plane && (const void*)x == (const void*)out) return hipErrorInvalidValue;
    switch (form) {
    case 0: return go_panel<T, 0>(a, x, y, out, tau, st);
    case 1: return go_panel<T, 1>(a, x, y, out, tau, st);
    case 2: return go_panel<T, 2>(a, x, y, out, tau, st);
    default: return hipErrorInvalidValue;
    }
}

template hipError_t launch_theta_panel<double>(const ThetaArgs&, const double*, const double*, double*,
                                               int, double, hipStream_t);
template hipError_t launch_theta_panel<float>(const ThetaArgs&, const float*, const float*, float*, int,
                                              double, hipStream_t);

}  // namespace wig2
