// Learned surrogate for the pair-interaction increment over a block of fine
// steps (the Theta[V12] part of the two-body operator, Sec. 3.1.2): a 4-D
// separable convolutional network on the phase-space grid, BF16 activations
// and weights on the bf16 matrix cores (v_mfma_f32_16x16x32_bf16, FP32
// accumulation), forward and backward.
//
// Input features (16 channels per grid point, from the block-start state
// f_t, zero off the p-box), in the form of the pair term, whose kernel is
// V12_m sin(2 pi m l / nx) on the antisymmetric differences along the
// anti-diagonal through the point (l = i1 - i2):
//   c_0 = s_in f_t(n1, n2)
//   c_m = s_in U sin(m a) [f_t(n1 - m, n2 + m) - f_t(n1 + m, n2 - m)],
//         m = 1..15, a = 2 pi l / nx, U = V12(0).
// Layers: h_0 = c; for each layer a one-dimensional convolution along one
// grid axis (p1, p2, x1, x2 in turn; K taps, 16 -> 16 channels; zero off the
// p-box, periodic in x) with a residual tanh,
//   h_{l+1} = h_l + tanh(b_l + sum_{t, c'} W_l[c][t][c'] h_l(P + (t - K/2) e_axis)[c']).
// Output: y = b_o + w_o . h_L + a . c (a linear path from the features),
// and the increment is Delta = s_out y.
//
// Every convolution runs on workgroup tiles of 32 positions along its axis
// times 16 grid points along a second axis, staged with the K - 1 halo
// positions in LDS (channel-last, 32 bytes per point); each wave contracts
// 8 positions: the A operand is the weight tile [16 c_out] x [2 taps x 16
// c_in], the B operand the staged input of those two taps at 16 points.  The
// input-gradient pass is the same convolution with the weights transposed
// and flipped (W^T[c'][K - 1 - t][c]); the weight-gradient pass stages both
// operands channel-major so that the contraction over points is the MFMA
// K dimension.
#include "common.h"

#include <algorithm>
#include <cmath>

namespace wig2 {
namespace {

constexpr int C = kSurC;   // channels
constexpr int TA = 32;     // output positions along the axis per tile
constexpr int NT = 256;    // threads per workgroup (4 waves x 8 positions)

typedef short s8v __attribute__((ext_vector_type(8)));
typedef float f4v __attribute__((ext_vector_type(4)));
typedef unsigned u4v __attribute__((ext_vector_type(4)));
typedef unsigned u2v __attribute__((ext_vector_type(2)));

__device__ inline unsigned short bf(float x)
{
    const unsigned u = __float_as_uint(x);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
__device__ inline float fb(unsigned short b)
{
    return __uint_as_float(((unsigned)b) << 16);
}

// Geometry of one tile: rest index r (two grid coordinates), segment of TA
// axis positions, block of 16 lane-axis points.
struct TileGeo {
    long base;  // point index of (rest, axis position 0, lane point 0)
    int a0;     // first output axis position of the tile
    int l0;     // first lane-axis point of the tile
};
__device__ inline TileGeo tile_geo(const SurAxis& g, long tile)
{
    const int nseg = (g.La + TA - 1) / TA, nlb = g.Ll / 16;
    TileGeo t;
    const int lb = (int)(tile % nlb);
    const long rs = tile / nlb;
    const int seg = (int)(rs % nseg);
    const long r = rs / nseg;
    t.base = (r / g.rdiv) * g.rs_hi + (r % g.rdiv) * g.rs_lo;
    t.a0 = seg * TA;
    t.l0 = lb * 16;
    return t;
}
__device__ inline long tiles_of(const SurAxis& g)
{
    return (long)g.R * ((g.La + TA - 1) / TA) * (g.Ll / 16);
}
// point index of axis position q (any integer) and lane point n, or -1 off
// the grid (non-periodic axis)
__device__ inline long point_at(const SurAxis& g, const TileGeo& t, int q, int n)
{
    if (g.periodic) {
        q %= g.La;
        if (q < 0) q += g.La;
    } else if (q < 0 || q >= g.La) {
        return -1;
    }
    return t.base + (long)q * g.Sa + (long)(t.l0 + n) * g.Sl;
}

// ---------------------------------------------------------------------------
// Convolution along one axis.  MODE 0: training forward (h -> t, h + t);
// MODE 1: input gradient (dh_next, t -> dz staged; dh = dh_next + conv^T dz);
// MODE 2: inference forward (h -> h + t).  wf: the layer's A fragments,
// [tap pair][lane][8] bf16 (transposed and flipped for MODE 1).
// ---------------------------------------------------------------------------
template <int MODE>
__global__ __launch_bounds__(NT) void k_sconv(SurAxis g, int K, const unsigned short* __restrict__ hin,
                                              const float* __restrict__ dhin, const unsigned short* __restrict__ tin,
                                              unsigned short* __restrict__ tout, unsigned short* __restrict__ hout,
                                              float* __restrict__ dhout, const unsigned short* __restrict__ wf,
                                              const float* __restrict__ bias)
{
    extern __shared__ unsigned char smem[];
    const int ntp = (K + 1) / 2;
    const int c = K / 2;
    const int rows = TA + 2 * ntp;  // staged positions a0 - c .. a0 + TA - 1 - c + 2 ntp
    unsigned short* S = reinterpret_cast<unsigned short*>(smem);            // [rows][16][16]
    unsigned short* Wl = S + (size_t)rows * 16 * C;                         // [ntp][64][8]
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int n = lane & 15, lk = lane >> 4;

    for (int e = tid; e < ntp * 64; e += NT)
        *reinterpret_cast<u4v*>(Wl + (size_t)e * 8) = *reinterpret_cast<const u4v*>(wf + (size_t)e * 8);
    const long ntiles = tiles_of(g);
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const TileGeo tg = tile_geo(g, tile);
        __syncthreads();  // the previous tile is done with S
        // stage rows: two threads per point, 8 channels (16 bytes) each
        for (int e = tid; e < rows * 32; e += NT) {
            const int a = e >> 5, pt = (e >> 1) & 15, hh = e & 1;
            const long P = point_at(g, tg, tg.a0 - c + a, pt);
            u4v v = {0u, 0u, 0u, 0u};
            if (P >= 0 && (tg.a0 - c + a < g.La || g.periodic)) {
                if constexpr (MODE == 1) {
                    // dz = dh_next (1 - t^2), rounded to bf16
                    const f4v d0 = *reinterpret_cast<const f4v*>(dhin + P * C + 8 * hh);
                    const f4v d1 = *reinterpret_cast<const f4v*>(dhin + P * C + 8 * hh + 4);
                    const u4v tv = *reinterpret_cast<const u4v*>(tin + P * C + 8 * hh);
                    unsigned short z[8];
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const unsigned word = tv[k >> 1];
                        const float tt = fb((unsigned short)((k & 1) ? (word >> 16) : (word & 0xFFFFu)));
                        const float dd = k < 4 ? d0[k] : d1[k - 4];
                        z[k] = bf(dd * (1.f - tt * tt));
                    }
#pragma unroll
                    for (int k = 0; k < 4; ++k) v[k] = (unsigned)z[2 * k] | ((unsigned)z[2 * k + 1] << 16);
                } else {
                    v = *reinterpret_cast<const u4v*>(hin + P * C + 8 * hh);
                }
            }
            *reinterpret_cast<u4v*>(S + ((size_t)a * 16 + pt) * C + 8 * hh) = v;
        }
        __syncthreads();
        f4v acc[8];
#pragma unroll
        for (int p = 0; p < 8; ++p) acc[p] = f4v{0.f, 0.f, 0.f, 0.f};
        for (int i = 0; i < ntp; ++i) {
            const s8v A = *reinterpret_cast<const s8v*>(Wl + ((size_t)i * 64 + lane) * 8);
            const int tap = 2 * i + (lk >> 1);
#pragma unroll
            for (int p = 0; p < 8; ++p) {
                const int row = 8 * w + p + tap;  // staged row of output position 8w + p, tap
                const s8v B = *reinterpret_cast<const s8v*>(S + ((size_t)row * 16 + n) * C + 8 * (lk & 1));
                acc[p] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[p], 0, 0, 0);
            }
        }
        // epilogue: lane holds c_out = 4 lk + j of point n at each position
#pragma unroll
        for (int p = 0; p < 8; ++p) {
            const int q = tg.a0 + 8 * w + p;
            if (q >= g.La) continue;
            const long P = tg.base + (long)q * g.Sa + (long)(tg.l0 + n) * g.Sl;
            if constexpr (MODE == 1) {
                const f4v d = *reinterpret_cast<const f4v*>(dhin + P * C + 4 * lk);
                *reinterpret_cast<f4v*>(dhout + P * C + 4 * lk) = d + acc[p];
            } else {
                const u2v hv = *reinterpret_cast<const u2v*>(S + ((size_t)(8 * w + p + c) * 16 + n) * C + 4 * lk);
                unsigned short to[4], ho[4];
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const unsigned word = hv[j >> 1];
                    const float h = fb((unsigned short)((j & 1) ? (word >> 16) : (word & 0xFFFFu)));
                    const float t = tanhf(acc[p][j] + bias[4 * lk + j]);
                    to[j] = bf(t);
                    ho[j] = bf(h + t);
                }
                const u2v hw = {(unsigned)ho[0] | ((unsigned)ho[1] << 16), (unsigned)ho[2] | ((unsigned)ho[3] << 16)};
                *reinterpret_cast<u2v*>(hout + P * C + 4 * lk) = hw;
                if constexpr (MODE == 0) {
                    const u2v tw = {(unsigned)to[0] | ((unsigned)to[1] << 16),
                                    (unsigned)to[2] | ((unsigned)to[3] << 16)};
                    *reinterpret_cast<u2v*>(tout + P * C + 4 * lk) = tw;
                }
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Weight gradient of one layer: dW[c][t][c'] = sum_P dz(P)[c] h(P + o_t)[c']
// and db[c] = sum_P dz(P)[c], dz = dh_next (1 - t^2).  Both operands are
// staged channel-major; wave w takes the taps t = w (mod 4), and wave 0 also
// the bias (a B operand of ones).  Per-workgroup sums go to part[wg][...].
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(NT) void k_sconv_dw(SurAxis g, int K, const unsigned short* __restrict__ hin,
                                                 const float* __restrict__ dhin, const unsigned short* __restrict__ tin,
                                                 float* __restrict__ part)
{
    extern __shared__ unsigned char smem[];
    const int c = K / 2;
    const int hrows = TA + K - 1;
    unsigned short* Z = reinterpret_cast<unsigned short*>(smem);  // dz^T [16][TA * 16]
    unsigned short* Hs = Z + (size_t)C * TA * 16;                 // h^T  [16][hrows * 16]
    const int tid = threadIdx.x, lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int m = lane & 15, lk = lane >> 4;
    constexpr int MAXT = 16;  // taps per wave (K <= 63)
    const int ntw = (K - w + 3) / 4;
    f4v acc[MAXT];
#pragma unroll
    for (int i = 0; i < MAXT; ++i) acc[i] = f4v{0.f, 0.f, 0.f, 0.f};
    f4v accb = {0.f, 0.f, 0.f, 0.f};
    const long ntiles = tiles_of(g);
    for (long tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        const TileGeo tg = tile_geo(g, tile);
        __syncthreads();
        // dz of the TA output positions (zero past the axis end)
        for (int e = tid; e < TA * 32; e += NT) {
            const int a = e >> 5, pt = (e >> 1) & 15, hh = e & 1;
            const int q = tg.a0 + a;
            float z[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
            if (q < g.La) {
                const long P = tg.base + (long)q * g.Sa + (long)(tg.l0 + pt) * g.Sl;
                const f4v d0 = *reinterpret_cast<const f4v*>(dhin + P * C + 8 * hh);
                const f4v d1 = *reinterpret_cast<const f4v*>(dhin + P * C + 8 * hh + 4);
                const u4v tv = *reinterpret_cast<const u4v*>(tin + P * C + 8 * hh);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const unsigned word = tv[k >> 1];
                    const float tt = fb((unsigned short)((k & 1) ? (word >> 16) : (word & 0xFFFFu)));
                    z[k] = (k < 4 ? d0[k] : d1[k - 4]) * (1.f - tt * tt);
                }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k) Z[(size_t)(8 * hh + k) * TA * 16 + a * 16 + pt] = bf(z[k]);
        }
        // h of positions a0 - c .. a0 + TA - 1 + c
        for (int e = tid; e < hrows * 32; e += NT) {
            const int a = e >> 5, pt = (e >> 1) & 15, hh = e & 1;
            const long P = point_at(g, tg, tg.a0 - c + a, pt);
            u4v v = {0u, 0u, 0u, 0u};
            if (P >= 0) v = *reinterpret_cast<const u4v*>(hin + P * C + 8 * hh);
#pragma unroll
            for (int k = 0; k < 8; ++k)
                Hs[(size_t)(8 * hh + k) * hrows * 16 + a * 16 + pt] =
                    (unsigned short)((k & 1) ? (v[k >> 1] >> 16) : (v[k >> 1] & 0xFFFFu));
        }
        __syncthreads();
        // k blocks of 32 (position, point) pairs: positions 2 kb + (lk >> 1),
        // points 8 (lk & 1) .. + 7
        for (int kb = 0; kb < TA / 2; ++kb) {
            const int a = 2 * kb + (lk >> 1), p0 = 8 * (lk & 1);
            const s8v A = *reinterpret_cast<const s8v*>(Z + (size_t)m * TA * 16 + a * 16 + p0);
#pragma unroll
            for (int i = 0; i < MAXT; ++i) {
                if (i < ntw) {  // wave-uniform
                    const int t = w + 4 * i;
                    const s8v B = *reinterpret_cast<const s8v*>(Hs + (size_t)m * hrows * 16 + (a + t) * 16 + p0);
                    acc[i] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[i], 0, 0, 0);
                }
            }
            if (w == 0) {
                const s8v ones = {0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80, 0x3F80};
                accb = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, ones, accb, 0, 0, 0);
            }
        }
    }
    // part[wg][c][t][c'] (c = 4 lk + j, c' = m) and part[wg][16 K + c]
    float* out = part + (size_t)blockIdx.x * (C * C * K + C);
#pragma unroll
    for (int i = 0; i < MAXT; ++i) {
        if (i < ntw) {
            const int t = w + 4 * i;
#pragma unroll
            for (int j = 0; j < 4; ++j) out[((size_t)(4 * lk + j) * K + t) * C + m] = acc[i][j];
        }
    }
    if (w == 0 && m == 0)
#pragma unroll
        for (int j = 0; j < 4; ++j) out[(size_t)C * C * K + 4 * lk + j] = accb[j];
}

// ---------------------------------------------------------------------------
// Features of the block-start state (16 channels, bf16).
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT) void k_sur_feat(const T* __restrict__ ft, int nx, int nk, long npts, SurScales sc,
                                                 unsigned short* __restrict__ feat)
{
    const long idx = (long)blockIdx.x * NT + threadIdx.x;
    if (idx >= npts) return;
    const int n2 = (int)(idx % nk), n1 = (int)((idx / nk) % nk);
    const long pl = idx / ((long)nk * nk);
    const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
    const int ell = (i1 - i2 + nx) % nx;
    const float ang = 6.283185307179586f * (float)ell / (float)nx;
    const float cs = sinf(ang), cc = cosf(ang);
    const T* F = ft + pl * (long)nk * nk;
    auto at = [&](int a, int b) { return (a >= 0 && a < nk && b >= 0 && b < nk) ? (float)F[(long)a * nk + b] : 0.f; };
    unsigned short z[C];
    z[0] = bf(sc.in_scale * at(n1, n2));
    float sm = cs, cm = cc;
#pragma unroll
    for (int mm = 1; mm < C; ++mm) {
        z[mm] = bf(sc.in_scale * sc.u_feat * sm * (at(n1 - mm, n2 + mm) - at(n1 + mm, n2 - mm)));
        const float sn = sm * cc + cm * cs;
        cm = cm * cc - sm * cs;
        sm = sn;
    }
    u4v* dst = reinterpret_cast<u4v*>(feat + idx * C);
    dst[0] = u4v{(unsigned)z[0] | ((unsigned)z[1] << 16), (unsigned)z[2] | ((unsigned)z[3] << 16),
                 (unsigned)z[4] | ((unsigned)z[5] << 16), (unsigned)z[6] | ((unsigned)z[7] << 16)};
    dst[1] = u4v{(unsigned)z[8] | ((unsigned)z[9] << 16), (unsigned)z[10] | ((unsigned)z[11] << 16),
                 (unsigned)z[12] | ((unsigned)z[13] << 16), (unsigned)z[14] | ((unsigned)z[15] << 16)};
}

// ---------------------------------------------------------------------------
// Output head y = b_o + w_o . h_L + a . c.  MODE 0: training (loss, dh_L
// and the head's gradient sums); MODE 1: loss only; MODE 2: inference
// f += s_out y.  head[] = {w_o[16], b_o, a[16]} (FP32).  Per-workgroup sums
// part[wg][33] (gradients) and lpart[wg] (sum of squared residuals).
// ---------------------------------------------------------------------------
template <typename T, int MODE>
__global__ __launch_bounds__(NT) void k_sur_head(const unsigned short* __restrict__ hL,
                                                 const unsigned short* __restrict__ feat, const T* __restrict__ delta,
                                                 T* __restrict__ f, long npts, SurScales sc,
                                                 const float* __restrict__ head, float gscale, float* __restrict__ dhL,
                                                 float* __restrict__ part, float* __restrict__ lpart)
{
    __shared__ float red[NT / 64][2 * C + 2];
    const long idx = (long)blockIdx.x * NT + threadIdx.x;
    const bool ok = idx < npts;
    float hv[C], cv[C];
    float y = head[C];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        hv[k] = ok ? fb(hL[idx * C + k]) : 0.f;
        cv[k] = ok ? fb(feat[idx * C + k]) : 0.f;
        y += head[k] * hv[k] + head[C + 1 + k] * cv[k];
    }
    if constexpr (MODE == 2) {
        if (ok) f[idx] = f[idx] + (T)(sc.out_scale * y);
        return;
    }
    const float r = ok ? y - sc.inv_out_scale * (float)delta[idx] : 0.f;
    const float dy = gscale * r;
    float vals[2 * C + 2];
#pragma unroll
    for (int k = 0; k < C; ++k) {
        vals[k] = dy * hv[k];
        vals[C + 1 + k] = dy * cv[k];
    }
    vals[C] = dy;
    vals[2 * C + 1] = r * r;
    if constexpr (MODE == 0) {
        if (ok) {
#pragma unroll
            for (int k = 0; k < C; k += 4)
                *reinterpret_cast<f4v*>(dhL + idx * C + k) =
                    f4v{dy * head[k], dy * head[k + 1], dy * head[k + 2], dy * head[k + 3]};
        }
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 2 * C + 2; ++k) {
        float v = vals[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        if (lane == 0) red[wv][k] = v;
    }
    __syncthreads();
    if (threadIdx.x < 2 * C + 2) {
        float s = 0.f;
        for (int k = 0; k < NT / 64; ++k) s += red[k][threadIdx.x];
        if (threadIdx.x == 2 * C + 1)
            lpart[blockIdx.x] = s;
        else if (MODE == 0)
            part[(size_t)blockIdx.x * (2 * C + 1) + threadIdx.x] = s;
    }
}

// grad[off + j] = scale * sum_w part[w][j], j < n (n values per workgroup)
__global__ void k_sur_reduce(const float* __restrict__ part, int nwg, int n, float scale, float* __restrict__ grad)
{
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    float s = 0.f;
    for (int w = 0; w < nwg; ++w) s += part[(size_t)w * n + j];
    grad[j] = scale * s;
}

// One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected).
__global__ void k_sur_adam(float* params, float* mom, float* var, const float* __restrict__ grad, long n, float lr,
                           int step)
{
    const long j = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    const float g = grad[j];
    const float b1 = 0.9f, b2 = 0.999f;
    const float m = b1 * mom[j] + (1.f - b1) * g;
    const float v = b2 * var[j] + (1.f - b2) * g * g;
    mom[j] = m;
    var[j] = v;
    const float mh = m / (1.f - powf(b1, (float)step));
    const float vh = v / (1.f - powf(b2, (float)step));
    params[j] -= lr * mh / (sqrtf(vh) + 1e-8f);
}

// A fragments of one layer from the FP32 weights W[c][t][c'] (t < K):
// frag[i][lane][e] = W[lane % 16][2 i + (lane / 16) / 2][8 ((lane / 16) % 2) + e]
// (forward), or the same of the transposed, flipped W^T[c'][K - 1 - t][c].
__global__ void k_sur_pack(const float* __restrict__ W, int K, int transposed, unsigned short* __restrict__ frag)
{
    const int ntp = (K + 1) / 2;
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ntp * 64 * 8) return;
    const int el = e % 8, lane = (e / 8) % 64, i = e / 512;
    const int row = lane % 16, lk = lane / 16;
    const int t = 2 * i + (lk >> 1), col = 8 * (lk & 1) + el;
    float v = 0.f;
    if (t < K) v = transposed ? W[((size_t)col * K + (K - 1 - t)) * C + row] : W[((size_t)row * K + t) * C + col];
    frag[e] = bf(v);
}

// d = a - b elementwise (T), and per-workgroup max|a - b| and max|b|.
template <typename T>
__global__ __launch_bounds__(NT) void k_diff_max(const T* a, const T* b, T* d, long n, float* part)
{
    __shared__ float r1[NT / 64], r2[NT / 64];
    float m1 = 0.f, m2 = 0.f;
    for (long i = (long)blockIdx.x * NT + threadIdx.x; i < n; i += (long)gridDim.x * NT) {
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
        for (int i = 1; i < NT / 64; ++i) {
            m1 = fmaxf(m1, r1[i]);
            m2 = fmaxf(m2, r2[i]);
        }
        part[2 * blockIdx.x] = m1;
        part[2 * blockIdx.x + 1] = m2;
    }
}

}  // namespace

size_t sur_conv_lds(int K)
{
    const int ntp = (K + 1) / 2;
    return (size_t)(TA + 2 * ntp) * 16 * C * 2 + (size_t)ntp * 64 * 8 * 2;
}
size_t sur_dw_lds(int K)
{
    return (size_t)C * TA * 16 * 2 + (size_t)C * (TA + K - 1) * 16 * 2;
}
long sur_tiles(const SurAxis& g)
{
    return (long)g.R * ((g.La + TA - 1) / TA) * (g.Ll / 16);
}

hipError_t launch_sur_conv(int mode, const SurAxis& g, int K, const unsigned short* hin, const float* dhin,
                           const unsigned short* tin, unsigned short* tout, unsigned short* hout, float* dhout,
                           const unsigned short* wf, const float* bias, int grid, hipStream_t st)
{
    const size_t sm = sur_conv_lds(K);
    const long nt = sur_tiles(g);
    const unsigned gr = (unsigned)std::min<long>(nt, grid);
    hipError_t e;
#define WIG2_SCONV(M)                                                                                        \
    e = hipFuncSetAttribute((const void*)k_sconv<M>, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);   \
    if (e != hipSuccess) return e;                                                                           \
    hipLaunchKernelGGL(k_sconv<M>, dim3(gr), dim3(NT), sm, st, g, K, hin, dhin, tin, tout, hout, dhout, wf, \
                       bias);
    if (mode == 0) {
        WIG2_SCONV(0)
    } else if (mode == 1) {
        WIG2_SCONV(1)
    } else {
        WIG2_SCONV(2)
    }
#undef WIG2_SCONV
    return hipGetLastError();
}

hipError_t launch_sur_dw(const SurAxis& g, int K, const unsigned short* hin, const float* dhin,
                         const unsigned short* tin, float* part, int grid, hipStream_t st)
{
    const size_t sm = sur_dw_lds(K);
    hipError_t e = hipFuncSetAttribute((const void*)k_sconv_dw, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_sconv_dw, dim3(grid), dim3(NT), sm, st, g, K, hin, dhin, tin, part);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sur_feat(const T* ft, int nx, int nk, const SurScales& sc, unsigned short* feat, hipStream_t st)
{
    const long npts = (long)nx * nx * nk * nk;
    hipLaunchKernelGGL(k_sur_feat<T>, dim3((unsigned)((npts + NT - 1) / NT)), dim3(NT), 0, st, ft, nx, nk, npts, sc,
                       feat);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_sur_head(int mode, const unsigned short* hL, const unsigned short* feat, const T* delta, T* f,
                           long npts, const SurScales& sc, const float* head, float gscale, float* dhL, float* part,
                           float* lpart, hipStream_t st)
{
    const unsigned nb = (unsigned)((npts + NT - 1) / NT);
    if (mode == 0)
        hipLaunchKernelGGL((k_sur_head<T, 0>), dim3(nb), dim3(NT), 0, st, hL, feat, delta, f, npts, sc, head, gscale,
                           dhL, part, lpart);
    else if (mode == 1)
        hipLaunchKernelGGL((k_sur_head<T, 1>), dim3(nb), dim3(NT), 0, st, hL, feat, delta, f, npts, sc, head, gscale,
                           dhL, part, lpart);
    else
        hipLaunchKernelGGL((k_sur_head<T, 2>), dim3(nb), dim3(NT), 0, st, hL, feat, delta, f, npts, sc, head, gscale,
                           dhL, part, lpart);
    return hipGetLastError();
}

hipError_t launch_sur_reduce(const float* part, int nwg, int n, float scale, float* grad, hipStream_t st)
{
    hipLaunchKernelGGL(k_sur_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, part, nwg, n, scale, grad);
    return hipGetLastError();
}

hipError_t launch_sur_adam(float* params, float* mom, float* var, const float* grad, long n, float lr, int step,
                           hipStream_t st)
{
    hipLaunchKernelGGL(k_sur_adam, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, params, mom, var, grad, n, lr,
                       step);
    return hipGetLastError();
}

hipError_t launch_sur_pack(const float* W, int K, int transposed, unsigned short* frag, hipStream_t st)
{
    const int n = (K + 1) / 2 * 64 * 8;
    hipLaunchKernelGGL(k_sur_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, W, K, transposed, frag);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_diff_max(const T* a, const T* b, T* d, long n, float* part, int nwg, hipStream_t st)
{
    hipLaunchKernelGGL(k_diff_max<T>, dim3(nwg), dim3(NT), 0, st, a, b, d, n, part);
    return hipGetLastError();
}
template hipError_t launch_diff_max<float>(const float*, const float*, float*, long, float*, int, hipStream_t);
template hipError_t launch_diff_max<double>(const double*, const double*, double*, long, float*, int,
                                            hipStream_t);

template hipError_t launch_sur_feat<float>(const float*, int, int, const SurScales&, unsigned short*, hipStream_t);
template hipError_t launch_sur_feat<double>(const double*, int, int, const SurScales&, unsigned short*, hipStream_t);
template hipError_t launch_sur_head<float>(int, const unsigned short*, const unsigned short*, const float*, float*,
                                           long, const SurScales&, const float*, float, float*, float*, float*,
                                           hipStream_t);
template hipError_t launch_sur_head<double>(int, const unsigned short*, const unsigned short*, const double*, double*,
                                            long, const SurScales&, const float*, float, float*, float*, float*,
                                            hipStream_t);

}  // namespace wig2
