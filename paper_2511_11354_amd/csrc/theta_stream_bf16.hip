// Split-BF16 streaming Theta for the torus (FP32 state) when the single-body
// symbols have a narrow band: the pair term (Sec. 3.1.2, eq. two_body_FSM) on
// the bf16 matrix cores with both operands split x = hi + lo
// (hi = RNE_bf16(x), lo = RNE_bf16(x - hi)), products hi*hi + hi*lo + lo*hi
// accumulated in FP32 on v_mfma_f32_16x16x32_bf16; the single-body
// differences (Sec. 3.1.1) on the vector ALUs from the same split plane.
//
// Same walk as the FP32 / FP64 streaming kernel: one persistent workgroup of
// NK/16 waves walks the planes, wave w owns the 16 rows n1 in [16w, 16w+16)
// and the skewed output tiles (n1, s = n1 + n2), and the next plane's loads
// are in flight during the second pass of the current one.
//
// LDS holds the plane split and skewed-transposed, H[s][k] = f(k, s - k)
// (zero where s - k is off the p-box), one 32-bit word per element holding
// its bf16 hi (low half) and lo (high half): the 8 consecutive k of one
// lane's B operand are two aligned 16-byte reads, separated into the hi and
// lo operands by byte permutes, and a single-body neighbour is one read.
// The Toeplitz A operand T[r][k] = sgn(r - k) kap(|r - k|) depends on r - k
// only, so its per-lane fragments [T(d - j)]_{j<8} are tabulated per plane
// for every d the tiles visit.  The kernel values are split three ways
// (hi + mid + lo, 24 bits, FP32's precision): the same kap enters every
// step, so a 16-bit kap would act as a slightly different pair potential
// whose effect grows with time; the products kept are
// kh xh + kh xl + km xh + km xl + kl xh.
//
// The split keeps the operator's structure: RNE-bf16 of -v is -RNE-bf16(v),
// so the split Toeplitz matrix is still skew and the plane sum of Theta x is
// still only the p-box edge leakage plus FP32 accumulation rounding.  What
// the split does change is kap itself, and kap enters every step: a 16-bit
// kap acts as a slightly different pair potential whose effect on the pair
// density grows with time, hence its 24-bit split.
#include "common.h"
#include "mfma.h"

#include <algorithm>

namespace wig2 {
namespace {
using namespace mf;

__device__ inline unsigned bf16_rne(float x)
{
    const unsigned u = __float_as_uint(x);
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}
__device__ inline float bf16_to_f(unsigned b)
{
    return __uint_as_float(b << 16);
}
// x = hi + lo for two values at once (v_cvt_pk_bf16_f32 rounds to nearest
// even): word k holds hi_k in its low half and lo_k in its high half
typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));
__device__ inline void split_pair2(float x0, float x1, unsigned& p0, unsigned& p1)
{
    const unsigned h = __builtin_bit_cast(unsigned, __builtin_convertvector((f2v{x0, x1}), b2v));
    const f2v r = {x0 - __uint_as_float(h << 16), x1 - __uint_as_float(h & 0xFFFF0000u)};
    const unsigned l = __builtin_bit_cast(unsigned, __builtin_convertvector(r, b2v));
    p0 = __builtin_amdgcn_perm(l, h, 0x05040100u);
    p1 = __builtin_amdgcn_perm(l, h, 0x07060302u);
}
// hi + lo of a packed (hi, lo) word as one bf16 dot product with (1, 1): both
// products are exact and hi + lo is representable in FP32, so this is the
// exact sum (up to the sign of a zero), one instruction instead of shift,
// mask and add
__device__ inline float pair_val(unsigned p)
{
    const b2v one = {(__bf16)1.0f, (__bf16)1.0f};
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(b2v, p), one, 0.0f, false);
}
// (a.hi + a.lo) - (b.hi + b.lo) as two dot products: the first is exact, the
// second rounds the exact difference once
__device__ inline float pair_diff(unsigned a, unsigned b)
{
    const b2v neg = {(__bf16)-1.0f, (__bf16)-1.0f};
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(b2v, b), neg, pair_val(a), false);
}

template <int NK>
struct B16Layout {
    static constexpr int NW = NK / 16;
    static constexpr int P = NK + 8;                   // row pitch (words): 8 zero columns per row
    static constexpr int ROWS0 = 5;                    // zero rows before s = 0
    static constexpr int ROWS = ROWS0 + 2 * NK + 4;    // s in [-5, 2 NK + 3]
    static constexpr int H_WORDS = ROWS * P;
    static constexpr int DMIN = -NK + 8;               // A fragments for d in [DMIN, NK - 1]
    static constexpr int NFR = NK - DMIN;
    static constexpr int KPT = 4;                      // fragment elements per thread
    static constexpr size_t bytes = 4 * (size_t)H_WORDS + 3 * 2 * 8 * (size_t)NFR;
    static_assert(8 * NFR <= KPT * NW * 64, "fragment table per thread");
    static_assert(P % 4 == 0, "16-byte rows");
};

template <int NK, bool TWO, int FORM>
__global__ __launch_bounds__(NK / 16 * 64) void k_theta_stream_bf16(
    const float* x, const float* y, float* out, int nx, long np, const double* __restrict__ sig1,
    const double* __restrict__ sig2, int band, const double* __restrict__ kap, double tau)
{
    typedef B16Layout<NK> L;
    typedef float f4v __attribute__((ext_vector_type(4)));
    typedef unsigned u4v __attribute__((ext_vector_type(4)));
    constexpr int NW = L::NW;
    constexpr int NT = NW * 64;
    constexpr int NS = NW + 1;  // skewed tiles per row block
    constexpr int P = L::P;
    constexpr int NV = NK * NK / (NT * 4);
    static_assert(NV == NW, "one 16 x 16 block of the plane per wave and round");

    extern __shared__ unsigned char smem_raw[];
    unsigned* H = reinterpret_cast<unsigned*>(smem_raw);
    unsigned short* Fr = reinterpret_cast<unsigned short*>(H + L::H_WORDS);  // [3][NFR][8]: hi, mid, lo

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int li = lane & 15, lk = lane >> 4;

    // everything outside the plane's support stays zero: the skewed corners,
    // the pad columns, the rows before s = 0 and after s = 2 NK - 2
    for (int e = tid; e < L::H_WORDS; e += NT) H[e] = 0u;
    long pl = blockIdx.x;
    if (pl >= np) return;  // whole workgroup leaves together
    const long stride = gridDim.x;

    auto Hat = [&](int s, int k) { return (s + L::ROWS0) * P + k; };

    // Plane loads: in round v wave w reads the 16 x 16 block
    // b = v NW + w (rows 16 (b / NW) + l % 16, columns 16 (b % NW) + 4 (l / 16)
    // .. + 3), so that the 16 lanes of a column group write 16 consecutive
    // rows of H in different LDS banks.
    f4v xr[NV];
    double kv[L::KPT];
    auto opaque_tid = [&]() {
        int t = tid;
        asm volatile("" : "+v"(t));
        return t;
    };
    auto fetch = [&](long p) {
        const float* src = x + p * (long)NK * NK;
        const int ot = opaque_tid(), ol = ot & 63;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int b = v * NW + w;
            const int n1 = 16 * (b / NW) + (ol & 15), n2 = 16 * (b % NW) + 4 * (ol >> 4);
            xr[v] = *reinterpret_cast<const f4v*>(src + (long)n1 * NK + n2);
        }
        if constexpr (TWO) {
            const int i1 = (int)(p / nx), i2 = (int)(p % nx);
            const int ell = (i1 - i2 + nx) % nx;
#pragma unroll
            for (int c = 0; c < L::KPT; ++c) {
                const int e = ot + c * NT;
                const int d = L::DMIN + e / 8 - (e % 8);
                const int ad = d < 0 ? -d : d;
                kv[c] = (e < 8 * L::NFR) ? kap[(long)ell * NK + min(max(ad, 1), NK - 1)] : 0.0;
            }
        }
    };

    // Lane-owned points: element q of tile j is n1 = 16 w + 4 lk + q,
    // s = 16 (w + j) + li, n2 = s - n1, valid when 0 <= n2 < NK.  Position
    // arithmetic restarts from an opaque copy of the lane id in each phase,
    // so the compiler cannot hoist the 4 NS per-point addresses and masks
    // out of the plane loop and keep them all live.
    auto opaque_lane = [&]() {
        int l = lane;
        asm volatile("" : "+v"(l));
        return l;
    };
    int el = opaque_lane();
    auto prow = [&](int q) { return 16 * w + 4 * (el >> 4) + q; };
    auto pcol = [&](int j, int q) { return 16 * (w + j) + (el & 15) - prow(q); };
    auto valid = [&](int j, int q) {
        const int n2 = pcol(j, q);
        return n2 >= 0 && n2 < NK;
    };

    // acc = pair term of the split plane in LDS at the lane-owned points
    auto pair_pass = [&](f4 (&acc)[NS]) {
#pragma unroll
        for (int j = 0; j < NS; ++j) acc[j] = f4{0.f, 0.f, 0.f, 0.f};
        if constexpr (TWO) {
#pragma unroll
            for (int KB = 0; KB < NK / 32; ++KB) {
                const int fi = (16 * w + li - 32 * KB - 8 * lk - L::DMIN) * 8;
                const s8 kh = *reinterpret_cast<const s8*>(Fr + fi);
                const s8 km = *reinterpret_cast<const s8*>(Fr + 8 * L::NFR + fi);
                const s8 kl = *reinterpret_cast<const s8*>(Fr + 16 * L::NFR + fi);
#pragma unroll
                for (int j = 0; j < NS; ++j) {
                    // tile s in [16(w+j), 16(w+j)+16), k in [32 KB, 32 KB + 32):
                    // some H[k][s] inside the p-box (wave-uniform test)
                    const int s0 = 16 * (w + j);
                    if (s0 + 15 < 32 * KB || s0 > 32 * KB + 31 + NK - 1) continue;
                    const u4v* src = reinterpret_cast<const u4v*>(H + Hat(s0 + li, 32 * KB + 8 * lk));
                    const u4v p0 = src[0], p1 = src[1];
                    const u4v bh = {__builtin_amdgcn_perm(p0[1], p0[0], 0x05040100u),
                                    __builtin_amdgcn_perm(p0[3], p0[2], 0x05040100u),
                                    __builtin_amdgcn_perm(p1[1], p1[0], 0x05040100u),
                                    __builtin_amdgcn_perm(p1[3], p1[2], 0x05040100u)};
                    const u4v bl = {__builtin_amdgcn_perm(p0[1], p0[0], 0x07060302u),
                                    __builtin_amdgcn_perm(p0[3], p0[2], 0x07060302u),
                                    __builtin_amdgcn_perm(p1[1], p1[0], 0x07060302u),
                                    __builtin_amdgcn_perm(p1[3], p1[2], 0x07060302u)};
                    const s8 xh = __builtin_bit_cast(s8, bh), xl = __builtin_bit_cast(s8, bl);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, xh, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kh, xl, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(km, xh, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(km, xl, acc[j], 0, 0, 0);
                    acc[j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(kl, xh, acc[j], 0, 0, 0);
                }
            }
        }
    };
    // acc += single-body differences of modes 1..band: for the lane's four
    // points (rows n1 = b + q, b = 16 w + 4 lk, on one anti-diagonal s),
    // f(n1, n2 -+ m) = H[s -+ m][n1] is one 16-byte read per side and
    // f(n1 -+ m, n2) = H[s -+ m][n1 -+ m] four word reads per side
    auto single_pass = [&](f4 (&acc)[NS], int i1, int i2) {
        for (int m = 1; m <= band; ++m) {
            el = opaque_lane();
            const float s1 = (float)sig1[(long)i1 * NK + m];
            const float s2 = (float)sig2[(long)i2 * NK + m];
            const int b = 16 * w + 4 * (el >> 4);
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const int s = 16 * (w + j) + (el & 15);
                const u4v lo2 = *reinterpret_cast<const u4v*>(H + Hat(s - m, b));
                const u4v hi2 = *reinterpret_cast<const u4v*>(H + Hat(s + m, b));
                const unsigned* lo1 = H + Hat(s - m, b - m);
                const unsigned* hi1 = H + Hat(s + m, b + m);
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const float d1 = pair_diff(lo1[q], hi1[q]);
                    const float d2 = pair_diff(lo2[q], hi2[q]);
                    acc[j][q] += s1 * d1 + s2 * d2;
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    fetch(pl);
    for (; pl < np; pl += stride) {
        const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
        const long pbase = pl * (long)NK * NK;
        {
            const int ot = opaque_tid(), ol = ot & 63;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int b = v * NW + w;
                const int n1 = 16 * (b / NW) + (ol & 15), n2 = 16 * (b % NW) + 4 * (ol >> 4);
                unsigned w0, w1, w2, w3;
                split_pair2(xr[v][0], xr[v][1], w0, w1);
                split_pair2(xr[v][2], xr[v][3], w2, w3);
                H[Hat(n1 + n2, n1)] = w0;
                H[Hat(n1 + n2 + 1, n1)] = w1;
                H[Hat(n1 + n2 + 2, n1)] = w2;
                H[Hat(n1 + n2 + 3, n1)] = w3;
            }
            if constexpr (TWO) {
#pragma unroll
                for (int c = 0; c < L::KPT; ++c) {
                    const int e = ot + c * NT;
                    if (e < 8 * L::NFR) {
                        const int d = L::DMIN + e / 8 - (e % 8);
                        const int ad = d < 0 ? -d : d;
                        // sgn(d) kap(|d|) = hi + mid + lo, each RNE-bf16 of the remainder
                        const double k = (ad > 0 && ad < NK) ? (d > 0 ? kv[c] : -kv[c]) : 0.0;
                        const unsigned h = bf16_rne((float)k);
                        const double r1 = k - (double)bf16_to_f(h);
                        const unsigned mm = bf16_rne((float)r1);
                        const unsigned l = bf16_rne((float)(r1 - (double)bf16_to_f(mm)));
                        Fr[e] = (unsigned short)h;
                        Fr[8 * L::NFR + e] = (unsigned short)mm;
                        Fr[16 * L::NFR + e] = (unsigned short)l;
                    }
                }
            }
        }
        __syncthreads();

        f4 acc[NS];
        pair_pass(acc);
        // the operand x at the lane-owned points (exact FP32, for the
        // epilogue; the plane has just been read, so these hit the cache),
        // in flight during the single-body pass
        float xv[NS][4];
        if constexpr (FORM != 0) {
            el = opaque_lane();
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int c = min(max(pcol(j, q), 0), NK - 1);
                    xv[j][q] = x[pbase + (long)prow(q) * NK + c];
                }
        }
        single_pass(acc, i1, i2);

        if constexpr (FORM == 0) {
            __syncthreads();  // every wave is done reading the plane
            if (pl + stride < np) fetch(pl + stride);
            el = opaque_lane();
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (valid(j, q)) out[pbase + (long)prow(q) * NK + pcol(j, q)] = acc[j][q];
            continue;
        }

        __syncthreads();  // every wave is done reading the plane

        if constexpr (FORM == 3) {
            // h = x + (tau/2) Theta x stays in registers; g = x + tau Theta x
            // replaces the plane in LDS
            float hv[NS][4];
            el = opaque_lane();
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                float g[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    hv[j][q] = xv[j][q] + (float)(0.5 * tau) * acc[j][q];
                    g[q] = xv[j][q] + (float)tau * acc[j][q];
                }
                unsigned gp[4];
                split_pair2(g[0], g[1], gp[0], gp[1]);
                split_pair2(g[2], g[3], gp[2], gp[3]);
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (valid(j, q)) H[Hat(16 * (w + j) + (el & 15), prow(q))] = gp[q];
            }
            __syncthreads();
            if (pl + stride < np) fetch(pl + stride);
            pair_pass(acc);
            single_pass(acc, i1, i2);
            el = opaque_lane();
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (valid(j, q))
                        out[pbase + (long)prow(q) * NK + pcol(j, q)] = hv[j][q] + (float)(0.5 * tau) * acc[j][q];
            __syncthreads();  // LDS plane is rewritten next
        } else {
            if (pl + stride < np) fetch(pl + stride);
            el = opaque_lane();
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if (!valid(j, q)) continue;
                    const long o = pbase + (long)prow(q) * NK + pcol(j, q);
                    const float th = acc[j][q];
                    if constexpr (FORM == 1)
                        out[o] = xv[j][q] + (float)tau * th;
                    else
                        out[o] = 0.5f * (y[o] + xv[j][q]) + (float)(0.5 * tau) * th;
                }
            __syncthreads();  // LDS plane is rewritten next
        }
    }
}

template <int NK, bool TWO, int FORM>
hipError_t go_bf16_stream(const ThetaArgs& a, const float* x, const float* y, float* out, double tau,
                          hipStream_t st)
{
    auto kf = k_theta_stream_bf16<NK, TWO, FORM>;
    const size_t sm = B16Layout<NK>::bytes;
    const int nt = NK / 16 * 64;
    hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    int dev = 0, ncu = 0, per = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kf, nt, sm)) != hipSuccess) return e;
    const long np = (long)a.nx * a.nx;
    const long grid = std::min<long>(np, (long)std::max(per, 1) * ncu);
    hipLaunchKernelGGL(kf, dim3((unsigned)grid), dim3(nt), sm, st, x, y, out, a.nx, np, a.sig1, a.sig2, a.band,
                       a.kap, tau);
    return hipGetLastError();
}

template <int NK, bool TWO>
hipError_t go_bf16_form(const ThetaArgs& a, const float* x, const float* y, float* out, int form, double tau,
                        hipStream_t st)
{
    switch (form) {
    case 0: return go_bf16_stream<NK, TWO, 0>(a, x, y, out, tau, st);
    case 1: return go_bf16_stream<NK, TWO, 1>(a, x, y, out, tau, st);
    case 2: return go_bf16_stream<NK, TWO, 2>(a, x, y, out, tau, st);
    case 3: return go_bf16_stream<NK, TWO, 3>(a, x, y, out, tau, st);
    default: return hipErrorInvalidValue;
    }
}

template <int NK>
hipError_t go_bf16_nk(const ThetaArgs& a, const float* x, const float* y, float* out, int form, double tau,
                      hipStream_t st)
{
    return a.kap ? go_bf16_form<NK, true>(a, x, y, out, form, tau, st)
                 : go_bf16_form<NK, false>(a, x, y, out, form, tau, st);
}

}  // namespace

bool theta_stream_bf16_ok(const ThetaArgs& a)
{
    return (a.nk == 32 || a.nk == 64 || a.nk == 96 || a.nk == 128) && !a.ksem && a.band >= 0 &&
           a.band <= kStreamBand && a.precision == WIG2_BF16X2;
}

hipError_t launch_theta_stream_bf16(const ThetaArgs& a, const float* x, const float* y, float* out, int form,
                                    double tau, hipStream_t st)
{
    if (!theta_stream_bf16_ok(a) || (form == 2 && !y)) return hipErrorNotSupported;
    switch (a.nk) {
    case 32: return go_bf16_nk<32>(a, x, y, out, form, tau, st);
    case 64: return go_bf16_nk<64>(a, x, y, out, form, tau, st);
    case 96: return go_bf16_nk<96>(a, x, y, out, form, tau, st);
    case 128: return go_bf16_nk<128>(a, x, y, out, form, tau, st);
    default: return hipErrorNotSupported;
    }
}

}  // namespace wig2
