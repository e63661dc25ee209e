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
// Operand layouts (16x16x4): lane l supplies A[l%16][l/16] and B[l/16][l%16];
// the accumulator row order differs between f32 and f64 (acc_row).
//
// Numerics: FP64 path on v_mfma_f64_16x16x4f64, FP32 path on
// v_mfma_f32_16x16x4f32, BF16X2 path on v_mfma_f32_16x16x32_bf16 with both
// operands split x = hi + lo (hi = RNE_bf16(x), lo = RNE_bf16(x - hi)) and
// hi*hi + hi*lo + lo*hi accumulated in FP32.  When the single-body symbols
// vanish beyond `band` modes (e.g. a few-mode V_ext), the single-body
// products only visit the k blocks within that band of each output tile.
#include "common.h"
#include "mfma.h"

#include <algorithm>

namespace wig2 {
namespace {

#ifndef WIG2_KEEP_H_ALWAYS
#define WIG2_KEEP_H_ALWAYS 0
#endif
using namespace mf;




// ---------------------------------------------------------------------------
// Products shared by the two-stage and the one-pass Heun plane bodies, on the
// plane X in LDS (pitch Plane<T, NK>::LD) and the signed Toeplitz tables.
// Operands of the next k-step are read from LDS while the matrix cores work
// on the current one (two register sets).
// ---------------------------------------------------------------------------
// acc += K1 X + X K2^T on the regular tiles of row block w (symbols vanishing
// beyond `band` modes; dense symbols take no per-instruction tests)
// PIPE = false (workgroups of more than 8 waves, 128 registers a wave, and
// the batched kernel, whose work-list loop leaves no room for the second
// register set): one register set, the k-step loop unrolled twice.
template <typename T, int NK, bool PIPE = true>
__device__ __forceinline__ void single_products(typename Acc<T>::V (&acc)[NK / 16], const T* X, const T* t1,
                                                const T* t2, int w, int li, int lk, int band)
{
    constexpr int NW = NK / 16;
    constexpr int LD = Plane<T, NK>::LD;
    const int r = 16 * w + li;
    if constexpr (!PIPE) {
        const int kb1_lo = max(0, 16 * w - band) / 4;
        const int kb1_hi = min(NK - 1, 16 * w + 15 + band) / 4;
        const T* pa1 = t1 + r + NK - lk;
        const T* pb1 = X + lk * LD + li;
#pragma unroll 2
        for (int kb = kb1_lo; kb <= kb1_hi; ++kb) {
            const T a1 = pa1[-4 * kb];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) acc[cb] = mma(a1, pb1[4 * kb * LD + 16 * cb], acc[cb]);
        }
        const T* pa2 = X + r * LD + lk;
        const T* pb2 = t2 + li + NK - lk;
#pragma unroll 2
        for (int kb = 0; kb < NK / 4; ++kb) {
            const T a2 = pa2[4 * kb];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) {
                if (4 * kb + 3 < 16 * cb - band || 4 * kb > 16 * cb + 15 + band) continue;
                acc[cb] = mma(a2, pb2[16 * cb - 4 * kb], acc[cb]);
            }
        }
        return;
    }
    T a[2], b[2][NW];
    auto mm = [&](int buf) {
#pragma unroll
        for (int cb = 0; cb < NW; ++cb) acc[cb] = mma(a[buf], b[buf][cb], acc[cb]);
    };
    // K1 X: K1[r][k] = t1[r - k + NK], rows within band of this wave
    const int kb1_lo = max(0, 16 * w - band) / 4;
    const int kb1_hi = min(NK - 1, 16 * w + 15 + band) / 4;
    const T* pa1 = t1 + r + NK - lk;
    const T* pb1 = X + lk * LD + li;
    auto ld1 = [&](int kb, int buf) {
        a[buf] = pa1[-4 * kb];
#pragma unroll
        for (int cb = 0; cb < NW; ++cb) b[buf][cb] = pb1[4 * kb * LD + 16 * cb];
    };
    int kb = kb1_lo;
    ld1(kb, 0);
    for (; kb + 1 <= kb1_hi; kb += 2) {
        ld1(kb + 1, 1);
        mm(0);
        __builtin_amdgcn_sched_barrier(0);
        if (kb + 2 <= kb1_hi) ld1(kb + 2, 0);
        mm(1);
        __builtin_amdgcn_sched_barrier(0);
    }
    if (kb <= kb1_hi) mm(0);
    // X K2^T: K2[c][k] = t2[c - k + NK]
    const T* pa2 = X + r * LD + lk;
    const T* pb2 = t2 + li + NK - lk;
    if (band >= NK - 1) {
        auto ld2 = [&](int k, int buf) {
            a[buf] = pa2[4 * k];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) b[buf][cb] = pb2[16 * cb - 4 * k];
        };
        ld2(0, 0);
        for (int k = 0; k < NK / 4; k += 2) {
            ld2(k + 1, 1);
            mm(0);
            __builtin_amdgcn_sched_barrier(0);
            if (k + 2 < NK / 4) ld2(k + 2, 0);
            mm(1);
            __builtin_amdgcn_sched_barrier(0);
        }
    } else {
#pragma unroll 2
        for (int k = 0; k < NK / 4; ++k) {
            const T a2 = pa2[4 * k];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb) {
                if (4 * k + 3 < 16 * cb - band || 4 * k > 16 * cb + 15 + band) continue;
                acc[cb] = mma(a2, pb2[16 * cb - 4 * k], acc[cb]);
            }
        }
    }
}

// sacc (+)= Theta_12 X on the skewed tiles (n1, s = n1 + n2) of row block w,
// over the k-block offset d = KB - w: the A operand depends on d alone and
// the tiles meeting k-block KB = w + d are j in [max(0, d), min(NW, d + NW)],
// fixed per d, so one wave-uniform test per k-block.  A = tk[r - k + NK],
// B = X[k LD + s - k] (zero gaps outside the plane).
template <typename T, int NK, bool PIPE = true>
__device__ __forceinline__ void pair_products(typename Acc<T>::V (&sacc)[NK / 16 + 1], const T* X, const T* tk,
                                              int w, int li, int lk)
{
    constexpr int NW = NK / 16;
    constexpr int NS = NW + 1;
    constexpr int LD = Plane<T, NK>::LD;
    if constexpr (!PIPE) {
        // per k-step, the tiles whose anti-diagonals meet its rows
        const T* pa = tk + 16 * w + li + NK - lk;
        const T* pb = X + lk * (LD - 1) + 16 * w + li;
#pragma unroll 2
        for (int kb = 0; kb < NK / 4; ++kb) {
            const T a = pa[-4 * kb];
#pragma unroll
            for (int j = 0; j < NS; ++j) {
                const int s0 = 16 * (w + j);
                if (4 * kb + 3 < s0 - NK + 1 || 4 * kb > s0 + 15) continue;  // wave-uniform
                sacc[j] = mma(a, pb[4 * kb * (LD - 1) + 16 * j], sacc[j]);
            }
        }
        return;
    }
    const T* pa0 = tk + li + NK - lk;
    const T* pb0 = X + lk * (LD - 1) + 16 * w * LD + li;
    T a[2], bv[2][NS];
#pragma unroll
    for (int d = -(NW - 1); d <= NW - 1; ++d) {
        if (w + d < 0 || w + d >= NW) continue;  // wave-uniform
        const int lo = d < 0 ? 0 : d, hi = d < 0 ? d + NW : NW;
        auto ldp = [&](int i, int buf) {
            a[buf] = pa0[-16 * d - 4 * i];
            const T* pb = pb0 + (16 * d + 4 * i) * (LD - 1);
#pragma unroll
            for (int j = 0; j < NS; ++j)
                if (j >= lo && j <= hi) bv[buf][j] = pb[16 * j];
        };
        ldp(0, 0);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int cur = i & 1;
            if (i + 1 < 4) ldp(i + 1, cur ^ 1);
#pragma unroll
            for (int j = 0; j < NS; ++j)
                if (j >= lo && j <= hi) sacc[j] = mma(a[cur], bv[cur][j], sacc[j]);
            __builtin_amdgcn_sched_barrier(0);
        }
    }
}

// ---------------------------------------------------------------------------
// FP64 / FP32 plane body.  One group of NK/16 waves handles one plane with
// its own LDS slice; several groups (planes) may share a workgroup.  Every
// thread of the workgroup calls the body with the same template arguments
// (inactive groups with active = false), so the barriers inside match.
// ---------------------------------------------------------------------------
template <typename T>
struct PlaneJob {
    const T* u;
    const T* v;
    T* out;
    long pl;  // plane index i1 * nx + i2
    int nx;
    const double* sig1;
    const double* sig2;
    const double* kap;
    const double* ksem;   // SEM matrices of particle 1 (box)
    const double* ksem2;  // of particle 2
    int band;
    double tau;
};

template <typename T, int NK, bool TWO, bool SEM, int MODE, bool PIPE>
__device__ __forceinline__ void theta_plane(const PlaneJob<T>& J, T* smem, int tid, bool active)
{
    typedef typename Acc<T>::V V;
    typedef Plane<T, NK> P;
    constexpr int NW = NK / 16;  // waves = row blocks
    constexpr int LD = P::LD;
    constexpr int NT = NW * 64;
    constexpr int NS = NW + 1;  // skewed tiles per row block

    const T* u = J.u;
    const T* __restrict__ vin = J.v;
    T* out = J.out;
    const int nx = J.nx, band = J.band;
    const double tau = J.tau;
    const double* __restrict__ sig1 = J.sig1;
    const double* __restrict__ sig2 = J.sig2;
    const double* __restrict__ kap = J.kap;
    const double* __restrict__ ksem = J.ksem;
    const double* __restrict__ ksem2 = J.ksem2;

    T* Xbase = smem;
    T* X = Xbase + kPadFront;            // X[r * LD + c]
    T* t1 = Xbase + P::X_ELEMS;          // t1[d + NK] = sgn(d) s1[|d|]
    T* t2 = t1 + P::TAB;                 // t2[d + NK] = sgn(d) s2[|d|]
    T* tk = t2 + P::TAB;                 // tk[d + NK] = sgn(d) kap[|d|]

    const long pl = J.pl;
    const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
    const int ell = (i1 - i2 + nx) % nx;
    const long pbase = pl * (long)NK * NK;

    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r = 16 * w + li;  // A-operand row of this lane
    constexpr bool KEEP_H = WIG2_KEEP_H_ALWAYS || !(sizeof(T) == 8 && NK >= 128 && TWO);
    T h[KEEP_H ? NW : 1][4];

    if (active) {
        for (int e = tid; e < 2 * NK; e += NT) {
            const int d = e - NK, ad = d < 0 ? -d : d;
            const bool ok = ad > 0 && ad < NK;
            t1[e] = (SEM || !ok) ? T(0) : sgnval(d, T(sig1[(long)i1 * NK + ad]));
            t2[e] = (SEM || !ok) ? T(0) : sgnval(d, T(sig2[(long)i2 * NK + ad]));
            tk[e] = (!TWO || !ok) ? T(0) : sgnval(d, T(kap[(long)ell * NK + ad]));
        }
        // zero gaps of the plane buffer
        for (int e = tid; e < kPadFront; e += NT) Xbase[e] = T(0);
        for (int e = tid; e < NK * kPadCols; e += NT) X[(e / kPadCols) * LD + NK + e % kPadCols] = T(0);

        // Each lane loads exactly the plane elements it later writes (the
        // accumulator layout): rows 16w + acc_row(lk, q), columns 16cb + li.
        // All loads are issued before the first use.  Stage 2 keeps
        // h = u + tau/2 v for its epilogue (u and v read once) unless that
        // would not fit the register file next to the accumulators; then the
        // epilogue reads u and v again.
        T xr[NW][4];
#pragma unroll
        for (int cb = 0; cb < NW; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                xr[cb][q] = u[pbase + (long)(16 * w + acc_row<T>(lk, q)) * NK + 16 * cb + li];
        if constexpr (MODE == 1) {
            T vr[NW][4];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    vr[cb][q] = vin[pbase + (long)(16 * w + acc_row<T>(lk, q)) * NK + 16 * cb + li];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    if constexpr (KEEP_H) h[cb][q] = xr[cb][q] + T(0.5 * tau) * vr[cb][q];
                    xr[cb][q] += T(tau) * vr[cb][q];
                }
        }
#pragma unroll
        for (int cb = 0; cb < NW; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                X[(16 * w + acc_row<T>(lk, q)) * LD + 16 * cb + li] = xr[cb][q];
    }
    __syncthreads();

    V acc[NW];
    V sacc[NS];
    if (active) {
    #pragma unroll
        for (int j = 0; j < NW; ++j) acc[j] = V{0, 0, 0, 0};

        if constexpr (SEM) {
            const double* K1 = ksem + (long)i1 * NK * NK;
            const double* K2 = ksem2 + (long)i2 * NK * NK;
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
            single_products<T, NK, PIPE>(acc, X, t1, t2, w, li, lk, band);
        }

        if constexpr (TWO) {
    #pragma unroll
            for (int j = 0; j < NS; ++j) sacc[j] = V{0, 0, 0, 0};
            pair_products<T, NK, PIPE>(sacc, X, tk, w, li, lk);
        }

    }
    __syncthreads();  // every wave is done reading the plane

    if constexpr (TWO) {
        if (active) {
            // scatter skewed tiles into the plane buffer: (n1, s) -> (n1, s - n1)
#pragma unroll
            for (int j = 0; j < NS; ++j) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int n1 = 16 * w + acc_row<T>(lk, q);
                    const int n2 = 16 * (w + j) + li - n1;
                    if (n2 >= 0 && n2 < NK) X[n1 * LD + n2] = sacc[j][q];
                }
            }
        }
        __syncthreads();
    }

    if (active) {
#pragma unroll
        for (int cb = 0; cb < NW; ++cb) {
            const int c = 16 * cb + li;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int rr = 16 * w + acc_row<T>(lk, q);
                T val = acc[cb][q];
                if constexpr (TWO) val += X[rr * LD + c];
                const long gi = pbase + (long)rr * NK + c;
                if constexpr (MODE == 0)
                    out[gi] = val;
                else if constexpr (KEEP_H)
                    out[gi] = h[cb][q] + T(0.5 * tau) * val;
                else
                    out[gi] = (u[gi] + T(0.5 * tau) * vin[gi]) + T(0.5 * tau) * val;
            }
        }
    }
    __syncthreads();  // the LDS slice may be reused by the next plane
}

// ---------------------------------------------------------------------------
// One-pass Heun step on the general kernel (torus, nk = 32 .. 128, dense or
// banded single-body symbols): out = f + (tau/2)(Theta f + Theta g), g = f +
// tau Theta f, with the potentials frozen over the step (Strang's sub-step), in
// one pass over the plane instead of the two stage launches, which read the
// state four times and write it twice.  Theta acts within the plane, so the
// plane stays in LDS between the two applications:
//   pass 1   regular tiles acc = K1 f + f K2^T, skewed tiles sacc = Theta_12 f;
//            sacc scattered into the LDS plane; at each lane's regular points
//            Theta f = acc + LDS, f re-read from the input;
//            FP64: acc = h = f + (tau/2) Theta f, LDS = (tau/2) g;
//            FP32: hv = h kept apart, LDS = g (accumulating onto h in FP32
//            rounds at the scale of f once per matrix-core instruction);
//   pass 2   the same products of the LDS plane (onto h in FP64), the pair
//            tiles scattered again, out = h + (tau/2) Theta g.
// out may alias f: every point is re-read and written by the same lane.
// ---------------------------------------------------------------------------
template <typename T, int NK, bool TWO>
__device__ __forceinline__ void theta_plane_heun(const PlaneJob<T>& J, T* smem, int tid)
{
    typedef typename Acc<T>::V V;
    typedef Plane<T, NK> P;
    constexpr int NW = NK / 16;
    constexpr int LD = P::LD;
    constexpr int NT = NW * 64;
    constexpr int NS = NW + 1;
    constexpr bool ONTO_H = sizeof(T) == 8;

    const T* u = J.u;
    T* out = J.out;
    const int nx = J.nx, band = J.band;
    const double tau = J.tau;
    const double* __restrict__ sig1 = J.sig1;
    const double* __restrict__ sig2 = J.sig2;
    const double* __restrict__ kap = J.kap;

    T* Xbase = smem;
    T* X = Xbase + kPadFront;
    T* t1 = Xbase + P::X_ELEMS;
    T* t2 = t1 + P::TAB;
    T* tk = t2 + P::TAB;

    const long pl = J.pl;
    const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
    const int ell = (i1 - i2 + nx) % nx;
    const long pbase = pl * (long)NK * NK;

    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r = 16 * w + li;

    for (int e = tid; e < 2 * NK; e += NT) {
        const int d = e - NK, ad = d < 0 ? -d : d;
        const bool ok = ad > 0 && ad < NK;
        t1[e] = !ok ? T(0) : sgnval(d, T(sig1[(long)i1 * NK + ad]));
        t2[e] = !ok ? T(0) : sgnval(d, T(sig2[(long)i2 * NK + ad]));
        tk[e] = (!TWO || !ok) ? T(0) : sgnval(d, T(kap[(long)ell * NK + ad]));
    }
    for (int e = tid; e < kPadFront; e += NT) Xbase[e] = T(0);
    for (int e = tid; e < NK * kPadCols; e += NT) X[(e / kPadCols) * LD + NK + e % kPadCols] = T(0);
    {
        T xr[NW][4];
#pragma unroll
        for (int cb = 0; cb < NW; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q)
                xr[cb][q] = u[pbase + (long)(16 * w + acc_row<T>(lk, q)) * NK + 16 * cb + li];
#pragma unroll
        for (int cb = 0; cb < NW; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) X[(16 * w + acc_row<T>(lk, q)) * LD + 16 * cb + li] = xr[cb][q];
    }
    __syncthreads();

    auto single = [&](V (&acc)[NW]) { single_products<T, NK>(acc, X, t1, t2, w, li, lk, band); };
    // sacc = Theta_12 X on the skewed tiles, then scattered into X once every
    // wave is done reading it
    auto pair_to_lds = [&](V (&sacc)[NS]) {
        if constexpr (TWO) {
#pragma unroll
            for (int j = 0; j < NS; ++j) sacc[j] = V{0, 0, 0, 0};
            pair_products<T, NK>(sacc, X, tk, w, li, lk);
        }
        __syncthreads();  // every wave is done reading the plane
        if constexpr (TWO) {
#pragma unroll
            for (int j = 0; j < NS; ++j)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const int n1 = 16 * w + acc_row<T>(lk, q);
                    const int n2 = 16 * (w + j) + li - n1;
                    if (n2 >= 0 && n2 < NK) X[n1 * LD + n2] = sacc[j][q];
                }
            __syncthreads();
        }
    };

    V acc[NW];
    V sacc[NS];
#pragma unroll
    for (int cb = 0; cb < NW; ++cb) acc[cb] = V{0, 0, 0, 0};
    single(acc);
    pair_to_lds(sacc);

    // pass-1 epilogue at the lane's regular points
    V hv[ONTO_H ? 1 : NW];
#pragma unroll
    for (int cb = 0; cb < NW; ++cb) {
        const int c = 16 * cb + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rr = 16 * w + acc_row<T>(lk, q);
            T th = acc[cb][q];
            if constexpr (TWO) th += X[rr * LD + c];
            const T fv = u[pbase + (long)rr * NK + c];
            if constexpr (ONTO_H) {
                acc[cb][q] = fv + T(0.5 * tau) * th;
                X[rr * LD + c] = T(0.5 * tau) * (fv + T(tau) * th);
            } else {
                hv[cb][q] = fv + T(0.5 * tau) * th;
                acc[cb][q] = T(0);
                X[rr * LD + c] = fv + T(tau) * th;
            }
        }
    }
    __syncthreads();

    single(acc);
    pair_to_lds(sacc);
#pragma unroll
    for (int cb = 0; cb < NW; ++cb) {
        const int c = 16 * cb + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int rr = 16 * w + acc_row<T>(lk, q);
            T th = acc[cb][q];
            if constexpr (TWO) th += X[rr * LD + c];
            const long gi = pbase + (long)rr * NK + c;
            if constexpr (ONTO_H)
                out[gi] = th;
            else
                out[gi] = hv[cb][q] + T(0.5 * tau) * th;
        }
    }
}

template <typename T, int NK, bool TWO>
__global__ __launch_bounds__(NK / 16 * 64) void k_theta_heun(const T* u, T* out, int nx, long np,
                                                            const double* __restrict__ sig1,
                                                            const double* __restrict__ sig2, int band,
                                                            const double* __restrict__ kap, double tau)
{
    extern __shared__ unsigned char smem_raw[];
    const long pl = blockIdx.x;
    if (pl >= np) return;  // whole workgroup leaves together
    PlaneJob<T> J{u, nullptr, out, pl, nx, sig1, sig2, kap, nullptr, nullptr, band, tau};
    theta_plane_heun<T, NK, TWO>(J, reinterpret_cast<T*>(smem_raw), threadIdx.x);
}

// Planes per workgroup for the single-context launch: small planes share a
// workgroup so that a workgroup has up to 8 waves.
template <int NK>
constexpr int planes_per_block()
{
    return (NK / 16 >= 8) ? 1 : (8 / (NK / 16) > 4 ? 4 : 8 / (NK / 16));
}

template <typename T, int NK, bool TWO, bool SEM, int MODE>
__global__ __launch_bounds__(NK / 16 * 64 * planes_per_block<NK>()) void k_theta(
    const T* u, const T* __restrict__ vin, T* out, int nx, long np, const double* __restrict__ sig1,
    const double* __restrict__ sig2, int band, const double* __restrict__ kap,
    const double* __restrict__ ksem, const double* __restrict__ ksem2, double tau)
{
    constexpr int NT = NK / 16 * 64;
    extern __shared__ unsigned char smem_raw[];
    const int g = threadIdx.x / NT;
    const long pl = (long)blockIdx.x * planes_per_block<NK>() + g;
    PlaneJob<T> J{u, vin, out, pl, nx, sig1, sig2, kap, ksem, ksem2, band, tau};
    T* smem = reinterpret_cast<T*>(smem_raw) + (size_t)g * (Plane<T, NK>::bytes / sizeof(T));
    theta_plane<T, NK, TWO, SEM, MODE, (NT * planes_per_block<NK>() <= 512)>(J, smem, threadIdx.x % NT, pl < np);
}


// ---------------------------------------------------------------------------
// Batched Theta: one persistent launch walks a list of (instance, planes)
// items over the whole ensemble.  Each item is workgroup-uniform, so all its
// waves run the same plane-size template; up to BLK/(64 NK/16) planes of the
// item share the workgroup, one LDS slice each.
// ---------------------------------------------------------------------------
template <typename T, int NK, int PB, int MODE>
__device__ __forceinline__ void theta_batch_item(const T* u_pool, const T* v_pool, T* out_pool,
                                                 const BatchInst& I, const ThItem& item,
                                                 const double* sig_pool, const double* kap_pool,
                                                 T* smem)
{
    constexpr int NT = NK / 16 * 64;
    const int g = threadIdx.x / NT;
    const bool active = g < item.np;
    PlaneJob<T> J{u_pool + I.off, v_pool ? v_pool + I.off : nullptr, out_pool + I.off,
                  (long)item.plane0 + g, I.nx, sig_pool + I.tab_off, sig_pool + I.tab_off,
                  kap_pool + I.tab_off, nullptr, nullptr, I.band, I.tau};
    T* slice = smem + (size_t)(active ? g : 0) * (Plane<T, NK>::bytes / sizeof(T));
    if (I.two_body)
        theta_plane<T, NK, true, false, MODE, false>(J, slice, threadIdx.x % NT, active);
    else
        theta_plane<T, NK, false, false, MODE, false>(J, slice, threadIdx.x % NT, active);
}

template <typename T, int NK, int PB, int MODE>
__global__ __launch_bounds__(NK / 16 * 64 * PB) void k_theta_batch(
    const T* u_pool, const T* v_pool, T* out_pool, const BatchInst* __restrict__ insts,
    const ThItem* __restrict__ items, int nitems, const double* __restrict__ sig_pool,
    const double* __restrict__ kap_pool)
{
    extern __shared__ unsigned char smem_raw[];
    T* smem = reinterpret_cast<T*>(smem_raw);
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const ThItem item = items[it];
        const BatchInst I = insts[item.inst];
        theta_batch_item<T, NK, PB, MODE>(u_pool, v_pool, out_pool, I, item, sig_pool, kap_pool, smem);
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
    const int lane = tid & 63, w = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int r = 16 * w + li;
    const int row0 = 16 * w + 4 * lk;
    float h[NW][4];
    {
        float xr[NW][4];
#pragma unroll
        for (int cb = 0; cb < NW; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) xr[cb][q] = u[pbase + (long)(row0 + q) * NK + 16 * cb + li];
        if constexpr (MODE == 1) {
            float vr[NW][4];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    vr[cb][q] = vin[pbase + (long)(row0 + q) * NK + 16 * cb + li];
#pragma unroll
            for (int cb = 0; cb < NW; ++cb)
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    h[cb][q] = xr[cb][q] + (float)(0.5 * tau) * vr[cb][q];
                    xr[cb][q] += (float)tau * vr[cb][q];
                }
        }
#pragma unroll
        for (int cb = 0; cb < NW; ++cb)
#pragma unroll
            for (int q = 0; q < 4; ++q) X[(row0 + q) * LD + 16 * cb + li] = xr[cb][q];
    }
    __syncthreads();

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
            if constexpr (MODE == 0)
                out[gi] = val;
            else
                out[gi] = h[cb][q] + (float)(0.5 * tau) * val;
        }
    }
}

template <typename T, int NK>
size_t smem_bytes_bf16()
{
    return sizeof(T) * ((size_t)NK * (NK + 1) + 3 * NK);
}

template <typename T, int NK, bool TWO, bool SEM>
hipError_t go(const ThetaArgs& a, const T* u, const T* v, T* out, int mode, double tau,
              hipStream_t st)
{
    const long np = (long)a.nx * a.nx;
    constexpr int PB = planes_per_block<NK>();
    const unsigned nb = (unsigned)((np + PB - 1) / PB);
    const size_t sm = Plane<T, NK>::bytes * PB;
    const int band = std::min(a.band, NK - 1);
    const dim3 blk(NK / 16 * 64 * PB);
    if (mode == 0) {
        auto kf = k_theta<T, NK, TWO, SEM, 0>;
        hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        hipLaunchKernelGGL(kf, dim3(nb), blk, sm, st, u, v, out, a.nx, np, a.sig1, a.sig2, band,
                           a.kap, a.ksem, a.ksem2 ? a.ksem2 : a.ksem, tau);
    } else {
        auto kf = k_theta<T, NK, TWO, SEM, 1>;
        hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
        hipLaunchKernelGGL(kf, dim3(nb), blk, sm, st, u, v, out, a.nx, np, a.sig1, a.sig2, band,
                           a.kap, a.ksem, a.ksem2 ? a.ksem2 : a.ksem, tau);
    }
    return hipGetLastError();
}

template <int NK, bool TWO>
hipError_t go_bf16(const ThetaArgs& a, const float* u, const float* v, float* out, int mode,
                   double tau, hipStream_t st)
{
    const unsigned np = (unsigned)((long)a.nx * a.nx);
    const size_t sm = smem_bytes_bf16<float, NK>();
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


// nk = 16 keeps the two stages: it is the plane size whose batched classes
// take the general kernel, and batched instances step bitwise as single
// contexts (the batched general kernel is the two-stage one).
bool theta_heun_general_ok(const ThetaArgs& a)
{
    const bool nk_ok = a.nk == 32 || a.nk == 48 || a.nk == 64 || a.nk == 96 || a.nk == 128;
    return nk_ok && !a.ksem && a.precision != WIG2_BF16X2;
}

namespace {
template <typename T, int NK>
hipError_t go_heun(const ThetaArgs& a, const T* x, T* out, double tau, hipStream_t st)
{
    const long np = (long)a.nx * a.nx;
    const size_t sm = Plane<T, NK>::bytes;
    const int band = std::min(a.band, NK - 1);
    auto kf = a.kap ? k_theta_heun<T, NK, true> : k_theta_heun<T, NK, false>;
    hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kf, dim3((unsigned)np), dim3(NK / 16 * 64), sm, st, x, out, a.nx, np, a.sig1, a.sig2,
                       band, a.kap, tau);
    return hipGetLastError();
}
}  // namespace

template <typename T>
hipError_t launch_theta_heun(const ThetaArgs& a, const T* x, T* out, double tau, hipStream_t st)
{
    if (!theta_heun_general_ok(a)) return hipErrorNotSupported;
    switch (a.nk) {
    case 32: return go_heun<T, 32>(a, x, out, tau, st);
    case 48: return go_heun<T, 48>(a, x, out, tau, st);
    case 64: return go_heun<T, 64>(a, x, out, tau, st);
    case 96: return go_heun<T, 96>(a, x, out, tau, st);
    default: return go_heun<T, 128>(a, x, out, tau, st);
    }
}
template hipError_t launch_theta_heun<double>(const ThetaArgs&, const double*, double*, double, hipStream_t);
template hipError_t launch_theta_heun<float>(const ThetaArgs&, const float*, float*, double, hipStream_t);

bool batch_nk_ok(int nk) { return nk == 16 || nk == 32 || nk == 48 || nk == 64 || nk == 96 || nk == 128; }

int batch_theta_max_planes(int nk, int elem_bytes)
{
    int p = 4;
    while (p > 1 && (nk / 16 * 64 * p > 1024 || batch_theta_lds(nk, p, elem_bytes) > 160 * 1024)) --p;
    return p;
}

size_t batch_theta_lds(int nk, int np, int elem_bytes)
{
    const size_t per = (size_t)elem_bytes * (kPadFront + (size_t)nk * (nk + kPadCols) + kPadCols + 6 * nk);
    return per * np;
}

namespace {
template <typename T, int NK, int PB>
hipError_t go_batch(const T* u, const T* v, T* o, const BatchInst* insts, const ThItem* items,
                    int nitems, int mode, const double* sig, const double* kap, int grid,
                    hipStream_t st)
{
    if constexpr (NK / 16 * 64 * PB > 1024) {
        return hipErrorInvalidValue;
    } else {
        const size_t lds = batch_theta_lds(NK, PB, sizeof(T));
        if (lds > 160 * 1024) return hipErrorInvalidValue;
        auto run = [&](auto kf) {
            hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
            hipLaunchKernelGGL(kf, dim3(grid), dim3(NK / 16 * 64 * PB), lds, st, u, v, o, insts, items,
                               nitems, sig, kap);
            return hipGetLastError();
        };
        return mode == 0 ? run(k_theta_batch<T, NK, PB, 0>) : run(k_theta_batch<T, NK, PB, 1>);
    }
}
template <typename T, int NK>
hipError_t go_batch_pb(int pb, const T* u, const T* v, T* o, const BatchInst* insts, const ThItem* items,
                       int nitems, int mode, const double* sig, const double* kap, int grid,
                       hipStream_t st)
{
    switch (pb) {
    case 1: return go_batch<T, NK, 1>(u, v, o, insts, items, nitems, mode, sig, kap, grid, st);
    case 2: return go_batch<T, NK, 2>(u, v, o, insts, items, nitems, mode, sig, kap, grid, st);
    case 3: return go_batch<T, NK, 3>(u, v, o, insts, items, nitems, mode, sig, kap, grid, st);
    case 4: return go_batch<T, NK, 4>(u, v, o, insts, items, nitems, mode, sig, kap, grid, st);
    default: return hipErrorInvalidValue;
    }
}
}  // namespace

template <typename T>
hipError_t launch_theta_batch(const T* u_pool, const T* v_pool, T* out_pool,
                              const BatchInst* insts, const ThItem* items, int nitems, int mode,
                              const double* sig_pool, const double* kap_pool, int nk, int planes,
                              int grid, hipStream_t st)
{
    if (nitems == 0) return hipSuccess;
    switch (nk) {
    case 16: return go_batch_pb<T, 16>(planes, u_pool, v_pool, out_pool, insts, items, nitems, mode, sig_pool, kap_pool, grid, st);
    case 32: return go_batch_pb<T, 32>(planes, u_pool, v_pool, out_pool, insts, items, nitems, mode, sig_pool, kap_pool, grid, st);
    case 48: return go_batch_pb<T, 48>(planes, u_pool, v_pool, out_pool, insts, items, nitems, mode, sig_pool, kap_pool, grid, st);
    case 64: return go_batch_pb<T, 64>(planes, u_pool, v_pool, out_pool, insts, items, nitems, mode, sig_pool, kap_pool, grid, st);
    case 96: return go_batch_pb<T, 96>(planes, u_pool, v_pool, out_pool, insts, items, nitems, mode, sig_pool, kap_pool, grid, st);
    case 128: return go_batch_pb<T, 128>(planes, u_pool, v_pool, out_pool, insts, items, nitems, mode, sig_pool, kap_pool, grid, st);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_theta_batch<double>(const double*, const double*, double*,
                                               const BatchInst*, const ThItem*, int, int,
                                               const double*, const double*, int, int, int,
                                               hipStream_t);
template hipError_t launch_theta_batch<float>(const float*, const float*, float*, const BatchInst*,
                                              const ThItem*, int, int, const double*,
                                              const double*, int, int, int, hipStream_t);

template hipError_t launch_theta<double>(const ThetaArgs&, const double*, const double*, double*,
                                         int, double, hipStream_t);
template hipError_t launch_theta<float>(const ThetaArgs&, const float*, const float*, float*, int,
                                        double, hipStream_t);

}  // namespace wig2
