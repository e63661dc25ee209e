// Theta on the torus by fast Fourier transforms (the FFT-accelerated route of
// the two-body cost statement in Sec. 3.1.2, with N >= 2 nk points per
// momentum direction as Sec. 3.1 sets the mesh up for).
//
// On a momentum plane (i1, i2) the three pseudo-difference terms of Sec. 3.1
// are linear convolutions of f(n1, n2) with odd kernels along the rows
// (particle 2's symbol s2), the columns (particle 1's s1) and the
// anti-diagonals (the pair kernel kap, shifting p1 and p2 in opposite
// directions).  Together they form one 2-D linear convolution.  Padding both
// momentum indices with zeros to N >= 2 nk (N = 2 nk rounded up to a
// multiple of 64) makes the cyclic convolution on the N x N torus equal to
// it on the nk x nk window, so
//   Theta f = IFFT2( W . FFT2(f) ),
//   W(k1, k2) = -2i [S1(k1) + S2(k2) + K((k1 - k2) mod N)],
//   S(k) = sum_{m >= 1} s_m sin(2 pi k m / N),
// which costs O(N^2 log N) per plane whatever the bands of the symbols are.
//
// One workgroup per plane.  No HBM workspace: the plane's 2-D spectrum is
// kept in LDS, half of it at a time for FP64 nk = 128.  The steps are:
//  * forward row transforms.  Rows 2r and 2r+1 are packed as the real and
//    imaginary parts of one complex row.
//  * per column frequency: unpack, forward column transform, multiply by W,
//    inverse column transform, repack.
//  * inverse row transforms.  The real and imaginary parts are again the
//    two rows.  Both halves add into registers.
// Each transform has N = 64 R points (R = 1, 1, 2, 2, 3, 4 for nk = 16, 32,
// 48, 64, 96, 128) and is done by one wavefront:
//  * the in-lane R-point DFT and its twiddles (four-step decomposition);
//  * a 64-point radix-2 transform across the lanes, by lane exchanges on
//    the vector ALUs (DPP moves and row / half swaps).
//  * Decimation in frequency: natural order in, bit-reversed out.
//  * Decimation in time: bit-reversed order in, natural order out.
// Lane orders are chosen so that every LDS access of a wave is consecutive.

#include "common.h"

namespace wig2 {
namespace {

template <typename T>
struct cx {
    T r, i;
};

template <typename T>
__device__ __forceinline__ cx<T> operator+(cx<T> a, cx<T> b) { return {a.r + b.r, a.i + b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator-(cx<T> a, cx<T> b) { return {a.r - b.r, a.i - b.i}; }
template <typename T>
__device__ __forceinline__ cx<T> operator*(cx<T> a, cx<T> b)
{
    return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename T>
__device__ __forceinline__ cx<T> conjg(cx<T> a) { return {a.r, -a.i}; }
template <typename T>
__device__ __forceinline__ cx<T> times_i(cx<T> a) { return {-a.i, a.r}; }
template <typename T>
__device__ __forceinline__ cx<T> times_mi(cx<T> a) { return {a.i, -a.r}; }

// Lane exchanges of the cross-lane stages.  The transforms index lanes by a
// logical number l; physical lane L holds l = (L & 0x38) | ((L ^ (L >> 1)) & 7),
// a linear map over GF(2) under which exchanging with l ^ 2^s is exchanging
// with L ^ m_s, m = (1, 3, 7, 15, 16, 32).  The first four are the DPP lane
// patterns quad_perm [1,0,3,2], quad_perm [3,2,1,0], row_half_mirror and
// row_mirror (vector-ALU moves).  For xor 16 and xor 32 the row and half
// swaps (v_permlane16_swap, v_permlane32_swap) give every lane both members
// of its pair (SWAP), so no exchange goes through the LDS crossbar, whose
// issue rate bounds the FP64 kernels at nk >= 64.  At nk = 128 (four
// sequences per lane, FP64 and FP32) the swaps trade a slot bit for the lane
// bit instead (register-transposed stages, no copies).  FP32 at nk <= 96 and
// FP64 at nk = 32, with more waves per SIMD and less vector-ALU headroom,
// keep ds_bpermute for those two stages (measured faster there than the
// copy-and-swap form).
__device__ __forceinline__ int logical_lane(int L) { return (L & 0x38) | ((L ^ (L >> 1)) & 7); }

template <int CTRL>
__device__ __forceinline__ int dpp_mov(int v)
{
    return __builtin_amdgcn_mov_dpp(v, CTRL, 0xF, 0xF, true);
}

template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v)
{
    const int lo = dpp_mov<CTRL>(__double2loint(v)), hi = dpp_mov<CTRL>(__double2hiint(v));
    return __hiloint2double(hi, lo);
}

template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v)
{
    return __int_as_float(dpp_mov<CTRL>(__float_as_int(v)));
}

// the value of logical lane l ^ 2^s (s is a constant after unrolling)
template <typename T>
__device__ __forceinline__ T xchg(T v, int s)
{
    switch (s) {
    case 0: return dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]: L ^ 1
    case 1: return dpp_mov<0x1B>(v);   // quad_perm [3,2,1,0]: L ^ 3
    case 2: return dpp_mov<0x141>(v);  // row_half_mirror: L ^ 7
    case 3: return dpp_mov<0x140>(v);  // row_mirror: L ^ 15
    case 4: return __shfl_xor(v, 16);
    default: return __shfl_xor(v, 32);
    }
}

template <typename T>
__device__ __forceinline__ cx<T> xchg_cx(cx<T> a, int s) { return {xchg(a.r, s), xchg(a.i, s)}; }

// Both members of the pair {L, L ^ 16} (S = 4) or {L, L ^ 32} (S = 5): lo is
// the value of the lane with the bit clear, hi of the lane with it set.
// Swapping the odd 16-lane rows (upper halves) of one copy with the even rows
// (lower halves) of another leaves the lower members in the first copy and
// the upper members in the second, in every lane.
template <int S>
__device__ __forceinline__ void pair_lohi(unsigned v, unsigned& lo, unsigned& hi)
{
    if constexpr (S == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        lo = r[0];
        hi = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        lo = r[0];
        hi = r[1];
    }
}

template <int S>
__device__ __forceinline__ void pair_lohi(double v, double& lo, double& hi)
{
    unsigned l0, h0, l1, h1;
    pair_lohi<S>((unsigned)__double2loint(v), l0, h0);
    pair_lohi<S>((unsigned)__double2hiint(v), l1, h1);
    lo = __hiloint2double((int)l1, (int)l0);
    hi = __hiloint2double((int)h1, (int)h0);
}

template <int S>
__device__ __forceinline__ void pair_lohi(float v, float& lo, float& hi)
{
    unsigned l, h;
    pair_lohi<S>(__float_as_uint(v), l, h);
    lo = __uint_as_float(l);
    hi = __uint_as_float(h);
}

// lo + sgn hi over the pair of stage s >= 4 (the lower lane's sum, the upper
// lane's difference)
template <int S, typename T>
__device__ __forceinline__ cx<T> pair_combine(cx<T> a, T sg)
{
    cx<T> lo, hi;
    pair_lohi<S>(a.r, lo.r, hi.r);
    pair_lohi<S>(a.i, lo.i, hi.i);
    return {fma(sg, hi.r, lo.r), fma(sg, hi.i, lo.i)};
}

// a t (CONJ: a conj(t))
template <bool CONJ, typename T>
__device__ __forceinline__ cx<T> cmul(cx<T> a, cx<T> t)
{
    if constexpr (CONJ)
        return {a.r * t.r + a.i * t.i, a.i * t.r - a.r * t.i};
    else
        return {a.r * t.r - a.i * t.i, a.r * t.i + a.i * t.r};
}

// Per-lane twiddles of the forward transform (the inverse uses conjugates).
// The cross-lane stage of span h = 2^s pairs lanes L and L + h (bit s of L
// clear); only the upper lane of a pair is multiplied by the twiddle, so the
// lower lane stores 1, and the sum / difference becomes y + sgn x, with
// sgn = +1 on the lower and -1 on the upper lane: no selects in the stages.
template <typename T, int R>
struct Twiddles {
    cx<T> stage[6];  // upper lane: e^{-i pi (lane mod h) / h}; lower lane: 1
    T sgn[6];
    cx<T> nat[R];    // e^{-2 pi i lane k1 / N}, k1 < R
    cx<T> rev[R];    // e^{-2 pi i br(lane) k1 / N}
    // the register-transposed stages (every lane): e^{-i pi (lane mod 16) / 16},
    // e^{-i pi (lane mod 32) / 32} and e^{-i pi (lane mod 16) / 32}
    cx<T> t4, t5, t5lo;
};

template <typename T, int R>
__device__ inline void make_twiddles(Twiddles<T, R>& w, int lane, int blane)
{
    constexpr int N = 64 * R;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        const int h = 1 << s;
        const bool upper = (lane & h) != 0;
        double sn, cs;
        sincospi(-(double)(lane & (h - 1)) / h, &sn, &cs);
        w.stage[s] = upper ? cx<T>{(T)cs, (T)sn} : cx<T>{T(1), T(0)};
        w.sgn[s] = upper ? T(-1) : T(1);
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        double sn, cs;
        sincospi(-2.0 * ((lane * k) % N) / N, &sn, &cs);
        w.nat[k] = {(T)cs, (T)sn};
        sincospi(-2.0 * ((blane * k) % N) / N, &sn, &cs);
        w.rev[k] = {(T)cs, (T)sn};
    }
    double sn, cs;
    sincospi(-(double)(lane & 15) / 16, &sn, &cs);
    w.t4 = {(T)cs, (T)sn};
    sincospi(-(double)(lane & 31) / 32, &sn, &cs);
    w.t5 = {(T)cs, (T)sn};
    sincospi(-(double)(lane & 15) / 32, &sn, &cs);
    w.t5lo = {(T)cs, (T)sn};
}

// 64-point transforms across the lanes, R independent sequences per lane.
// Decimation in frequency: lane L ends with element br(L).
// Lower lane: x + y; upper lane: (y - x) t.
template <bool INV, bool SWAP, typename T, int R, int SHI = 5>
__device__ __forceinline__ void dif64(cx<T> (&x)[R], const Twiddles<T, R>& w)
{
#pragma unroll
    for (int s = SHI; s >= 0; --s) {
        const T sg = w.sgn[s];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            cx<T> d;
            if (SWAP && s >= 4) {
                d = s == 4 ? pair_combine<4>(x[k], sg) : pair_combine<5>(x[k], sg);
            } else {
                const cx<T> y = xchg_cx(x[k], s);
                d = {fma(sg, x[k].r, y.r), fma(sg, x[k].i, y.i)};
            }
            x[k] = s == 0 ? d : cmul<INV>(d, w.stage[s]);
        }
    }
}

// Decimation in time: lane L starts with element br(L), ends with element L.
// Lower lane: x + t y; upper lane: y - t x (the upper lane's value is
// multiplied by t before the exchange).
template <bool INV, bool SWAP, typename T, int R, int SEND = 6>
__device__ __forceinline__ void dit64(cx<T> (&x)[R], const Twiddles<T, R>& w)
{
#pragma unroll
    for (int s = 0; s < SEND; ++s) {
        const T sg = w.sgn[s];
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const cx<T> m = s == 0 ? x[k] : cmul<INV>(x[k], w.stage[s]);
            if (SWAP && s >= 4) {
                x[k] = s == 4 ? pair_combine<4>(m, sg) : pair_combine<5>(m, sg);
            } else {
                const cx<T> o = xchg_cx(m, s);
                x[k] = {fma(sg, m.r, o.r), fma(sg, m.i, o.i)};
            }
        }
    }
}

// In-lane part of a forward transform whose input is zero past the plane
// (x[a] = 0 for 64 a >= nk = N/2: a >= 1 at R = 2, a >= 2 at R = 3, 4):
// x[a] -> DFT_R over a, times the twiddles.
template <typename T, int R>
__device__ __forceinline__ void fwd_inlane(cx<T> (&x)[R], const cx<T> (&tw)[R])
{
    constexpr T h3 = T(0.86602540378443864676);  // sin(pi/3)
    if constexpr (R == 2) {
        x[1] = x[0] * tw[1];
    } else if constexpr (R == 3) {
        const cx<T> a = x[0], b = x[1];
        const cx<T> c = {a.r - T(0.5) * b.r, a.i - T(0.5) * b.i};  // a - b/2
        const cx<T> e = {h3 * b.r, h3 * b.i};                        // (sqrt 3 / 2) b
        x[0] = a + b;
        x[1] = (c + times_mi(e)) * tw[1];
        x[2] = (c + times_i(e)) * tw[2];
    } else if constexpr (R == 4) {
        const cx<T> a = x[0], b = x[1];
        x[0] = a + b;
        x[1] = (a + times_mi(b)) * tw[1];
        x[2] = (a - b) * tw[2];
        x[3] = (a + times_i(b)) * tw[3];
    }
}

// In-lane part of an inverse transform of which only the plane's positions
// are kept (64 a < nk): conjugate twiddles, then the inverse DFT_R into
// x[0 .. NA).
template <typename T, int R>
__device__ __forceinline__ void inv_inlane(cx<T> (&z)[R], const cx<T> (&tw)[R])
{
    constexpr T h3 = T(0.86602540378443864676);
#pragma unroll
    for (int k = 1; k < R; ++k) z[k] = z[k] * conjg(tw[k]);
    if constexpr (R == 2) {
        z[0] = z[0] + z[1];
    } else if constexpr (R == 3) {
        const cx<T> s12 = z[1] + z[2], d12 = z[1] - z[2];
        const cx<T> c0 = z[0] + s12;
        const cx<T> c1 = cx<T>{z[0].r - T(0.5) * s12.r, z[0].i - T(0.5) * s12.i} +
                         times_i(cx<T>{h3 * d12.r, h3 * d12.i});
        z[0] = c0;
        z[1] = c1;
    } else if constexpr (R == 4) {
        const cx<T> c0 = (z[0] + z[2]) + (z[1] + z[3]);
        const cx<T> c1 = (z[0] - z[2]) + times_i(z[1] - z[3]);
        z[0] = c0;
        z[1] = c1;
    }
}

// Register-transposed stages for four sequences per lane (R = 4).  A row
// swap of registers a and b (v_permlane16_swap for lane bit 4, S = 4, or
// v_permlane32_swap for lane bit 5, S = 5) leaves in every lane both members
// of a pair of lanes: a holds the lower member (bit clear), b the upper.
// The sequence they belong to is now given by the lane bit, and the
// butterfly runs in registers with a useful twiddle in every lane.  A
// transform whose last two stages are done this way ends "transposed": slot k
// holds positions with bit 4 = k >> 1 and bit 5 = k & 1, and lane bits 5, 4
// give the in-lane index k1 = bit5 | bit4 << 1.  swap_rows moves a slot bit
// back into its lane bit.
template <int S>
__device__ __forceinline__ void swap_rows(unsigned& a, unsigned& b)
{
    if constexpr (S == 4) {
        const auto r = __builtin_amdgcn_permlane16_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    } else {
        const auto r = __builtin_amdgcn_permlane32_swap(a, b, false, false);
        a = r[0];
        b = r[1];
    }
}

template <int S>
__device__ __forceinline__ void swap_rows(double& a, double& b)
{
    unsigned al = (unsigned)__double2loint(a), ah = (unsigned)__double2hiint(a);
    unsigned bl = (unsigned)__double2loint(b), bh = (unsigned)__double2hiint(b);
    swap_rows<S>(al, bl);
    swap_rows<S>(ah, bh);
    a = __hiloint2double((int)ah, (int)al);
    b = __hiloint2double((int)bh, (int)bl);
}

template <int S>
__device__ __forceinline__ void swap_rows(float& a, float& b)
{
    unsigned au = __float_as_uint(a), bu = __float_as_uint(b);
    swap_rows<S>(au, bu);
    a = __uint_as_float(au);
    b = __uint_as_float(bu);
}

template <int S, typename T>
__device__ __forceinline__ void swap_rows(cx<T>& a, cx<T>& b)
{
    swap_rows<S>(a.r, b.r);
    swap_rows<S>(a.i, b.i);
}

// decimation in time, bit-reversed standard input, transposed output
template <bool INV, typename T>
__device__ __forceinline__ void dit64_to_trx(cx<T> (&x)[4], const Twiddles<T, 4>& w)
{
    dit64<INV, false, T, 4, 4>(x, w);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        swap_rows<4>(x[k], x[k + 2]);
        const cx<T> m = cmul<INV>(x[k + 2], w.t4), lo = x[k];
        x[k] = lo + m;
        x[k + 2] = lo - m;
    }
    // position bit 4 now sits in slot bit 1: its twiddle factor e^{-i pi/2}
    // (conjugated for the inverse) multiplies the pair (2, 3)
#pragma unroll
    for (int k = 0; k < 4; k += 2) {
        swap_rows<5>(x[k], x[k + 1]);
        cx<T> m = cmul<INV>(x[k + 1], w.t5lo);
        if (k == 2) m = INV ? times_i(m) : times_mi(m);
        const cx<T> lo = x[k];
        x[k] = lo + m;
        x[k + 1] = lo - m;
    }
}

// decimation in frequency, natural standard input, transposed output
template <bool INV, typename T>
__device__ __forceinline__ void dif64_to_trx(cx<T> (&x)[4], const Twiddles<T, 4>& w)
{
#pragma unroll
    for (int k = 0; k < 4; k += 2) {
        swap_rows<5>(x[k], x[k + 1]);
        const cx<T> lo = x[k], hi = x[k + 1];
        x[k] = lo + hi;
        x[k + 1] = cmul<INV>(lo - hi, w.t5);
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        swap_rows<4>(x[k], x[k + 2]);
        const cx<T> lo = x[k], hi = x[k + 2];
        x[k] = lo + hi;
        x[k + 2] = cmul<INV>(lo - hi, w.t4);
    }
    dif64<INV, false, T, 4, 3>(x, w);
}

// decimation in time, transposed input (as dif64_to_trx leaves it),
// natural standard output
template <bool INV, typename T>
__device__ __forceinline__ void dit64_from_trx(cx<T> (&x)[4], const Twiddles<T, 4>& w)
{
    dit64<INV, false, T, 4, 4>(x, w);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const cx<T> m = cmul<INV>(x[k + 2], w.t4), lo = x[k];
        x[k] = lo + m;
        x[k + 2] = lo - m;
        swap_rows<4>(x[k], x[k + 2]);
    }
#pragma unroll
    for (int k = 0; k < 4; k += 2) {
        const cx<T> m = cmul<INV>(x[k + 1], w.t5), lo = x[k];
        x[k] = lo + m;
        x[k + 1] = lo - m;
        swap_rows<5>(x[k], x[k + 1]);
    }
}

// decimation in frequency, transposed input, bit-reversed standard output
template <bool INV, typename T>
__device__ __forceinline__ void dif64_from_trx(cx<T> (&x)[4], const Twiddles<T, 4>& w)
{
#pragma unroll
    for (int k = 0; k < 4; k += 2) {
        const cx<T> lo = x[k], hi = x[k + 1];
        cx<T> m = cmul<INV>(lo - hi, w.t5lo);
        if (k == 2) m = INV ? times_i(m) : times_mi(m);
        x[k] = lo + hi;
        x[k + 1] = m;
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const cx<T> lo = x[k], hi = x[k + 2];
        x[k] = lo + hi;
        x[k + 2] = cmul<INV>(lo - hi, w.t4);
    }
    dif64<INV, false, T, 4, 3>(x, w);
#pragma unroll
    for (int k = 0; k < 2; ++k) swap_rows<4>(x[k], x[k + 2]);
#pragma unroll
    for (int k = 0; k < 4; k += 2) swap_rows<5>(x[k], x[k + 1]);
}

// Wavefronts per workgroup: nk/16 (eight row pairs each); FP32 at nk >= 64
// takes twice as many (four row pairs each: 51-75 VGPRs, more waves to hide
// the exchange and LDS latency; measured 3-27% faster there, 6% slower at
// nk = 32), FP64 at nk = 96 eight (six row pairs each: two waves on every
// SIMD instead of one or two; 17% faster).  FP64 at nk = 128 has no
// register room for more.
template <typename T, int NK>
constexpr int fft_waves()
{
    if (sizeof(T) == 8 && NK == 96) return 8;
    return (sizeof(T) == 4 && NK >= 64 ? 2 : 1) * NK / 16;
}

template <typename T, int NK>
struct FftShape {
    static constexpr int N = fft_len(NK);       // padded length
    static constexpr int R = N / 64;            // values per lane
    static constexpr int P = (sizeof(T) == 8 && NK == 128) ? 2 : 1;  // spectrum passes
    static constexpr int NJ = R / P;            // in-lane indices k1 per pass (k1 = p + P jj)
    static constexpr int NW = fft_waves<T, NK>();  // wavefronts
    static constexpr int RPW = NK / 2 / NW;     // row pairs per wavefront
    static constexpr int NA = (NK + 63) / 64;   // in-lane positions inside the window
    static constexpr int PITCH = NJ * 64 + 1;   // complex values per row pair in LDS
    static constexpr bool SWAP = sizeof(T) == 8 && NK >= 64;  // lane swaps for xor 16 / 32
    static constexpr bool TRX = R == 4;  // register-transposed swap stages (nk = 128)
    static constexpr size_t lds() { return sizeof(cx<T>) * (NK / 2) * PITCH + sizeof(T) * 3 * N; }
};

// Plane symbols: sym[(w nx + row) N + k] = S_w(k) / N^2 for w = 0 (s1, row
// i1), 1 (s2, row i2), 2 (kap, row (i1 - i2) mod nx), N = fft_len(nk).  The
// 1/N^2 is the normalisation of the two inverse transforms.
__global__ void __launch_bounds__(256) k_fft_symbols(int nx, int nk, const double* __restrict__ sig1,
                                                    const double* __restrict__ sig2,
                                                    const double* __restrict__ kap, double* __restrict__ sym)
{
    __shared__ double sn[2 * kMaxThetaNk];
    __shared__ double sv[kMaxThetaNk];
    const int N = fft_len(nk), row = blockIdx.x, which = blockIdx.y;
    const double* s = which == 0 ? sig1 : which == 1 ? sig2 : kap;
    for (int t = threadIdx.x; t < N; t += blockDim.x) sn[t] = sinpi(2.0 * t / N);
    for (int t = threadIdx.x; t < nk; t += blockDim.x) sv[t] = s ? s[(long)row * nk + t] : 0.0;
    __syncthreads();
    const double scale = 1.0 / ((double)N * N);
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        double acc = 0.0;
        for (int m = 1; m < nk; ++m) acc += sv[m] * sn[(k * m) % N];
        sym[((long)which * nx + row) * N + k] = acc * scale;
    }
}

// out = alpha Theta (u + beta v) + cu u + cv v on plane blockIdx.x; out may
// be u (every read of the plane precedes its writes, all in this workgroup).
template <typename T, int NK>
__global__ void __launch_bounds__((fft_waves<T, NK>() * 64)) k_theta_fft(int nx, const double* __restrict__ sym, const T* u,
                                                           const T* v, T* out, T beta, T alpha, T cu, T cv)
{
    using S = FftShape<T, NK>;
    constexpr int N = S::N, R = S::R, P = S::P, NJ = S::NJ, RPW = S::RPW, NA = S::NA, PITCH = S::PITCH;
    constexpr bool SW = S::SWAP, TRX = S::TRX;
    extern __shared__ unsigned char smem_raw[];
    cx<T>* A = reinterpret_cast<cx<T>*>(smem_raw);
    T* tab = reinterpret_cast<T*>(A + (NK / 2) * PITCH);  // S1 | S2 | K, N each

    const int lane = logical_lane(threadIdx.x & 63), wave = threadIdx.x >> 6;
    const int blane = (int)(__builtin_bitreverse32((unsigned)lane) >> 26);
    const long plane = blockIdx.x;
    const int i1 = (int)(plane / nx), i2 = (int)(plane % nx), ell = (i1 - i2 + nx) % nx;
    const long pbase = plane * NK * NK;
    const bool with_v = v != nullptr && beta != T(0);
    const bool add_base = cu != T(0) || cv != T(0);

    for (int t = threadIdx.x; t < 3 * N; t += blockDim.x) {
        const int w = t / N, k = t - w * N;
        const int row = w == 0 ? i1 : w == 1 ? i2 : ell;
        tab[t] = (T)sym[((long)w * nx + row) * N + k];
    }
    Twiddles<T, R> tw;
    make_twiddles(tw, lane, blane);

    cx<T> acc[RPW][NA];
#pragma unroll
    for (int q = 0; q < RPW; ++q)
#pragma unroll
        for (int a = 0; a < NA; ++a) acc[q][a] = {T(0), T(0)};

#pragma unroll
    for (int p = 0; p < P; ++p) {  // unrolled: p selects register-array entries
        // forward row transforms: lane L loads n2 = 64a + br(L), holds Z[k1 + R L]
        // after; the next row pair's values are loaded during this transform
        cx<T> ru[NA], rv[NA];
        auto load_rows = [&](int r) {
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int n2 = 64 * a + blane;
                ru[a] = rv[a] = {T(0), T(0)};
                if (n2 < NK) {
                    const long i0 = pbase + (long)(2 * r) * NK + n2;
                    ru[a] = {u[i0], u[i0 + NK]};
                    if (with_v) rv[a] = {v[i0], v[i0 + NK]};
                }
            }
        };
        load_rows(wave * RPW);
#pragma unroll 1
        for (int q = 0; q < RPW; ++q) {
            const int r = wave * RPW + q;
            cx<T> x[R];
#pragma unroll
            for (int a = 0; a < R; ++a) {
                x[a] = {T(0), T(0)};
                if (a < NA) x[a] = with_v ? cx<T>{fma(beta, rv[a].r, ru[a].r), fma(beta, rv[a].i, ru[a].i)} : ru[a];
            }
            if (q + 1 < RPW) load_rows(r + 1);
            fwd_inlane(x, tw.rev);
            if constexpr (TRX) {
                // transposed: lane bits 5, 4 carry k1, the slots position bits 5, 4;
                // this pass keeps k1 = p + P jj
                dit64_to_trx<false>(x, tw);
                const int k1l = ((lane >> 5) & 1) | (((lane >> 4) & 1) << 1);
                if (k1l % P == p) {
                    const int jj = k1l / P;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        A[r * PITCH + jj * 64 + ((lane & 15) | ((k >> 1) << 4) | ((k & 1) << 5))] = x[k];
                }
            } else {
                dit64<false, SW>(x, tw);
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) A[r * PITCH + jj * 64 + lane] = x[p + P * jj];
            }
        }
        __syncthreads();

        // column frequencies k2 = p + P c in [0, N/2]; k2 and N - k2 share a job
        const int ncol = (N / 2 - p) / P + 1;
        const T* S1 = tab;
        const T* S2 = tab + N;
        const T* KK = tab + 2 * N;
#pragma unroll 1
        for (int c = wave; c < ncol; c += S::NW) {
            const int k2 = p + P * c, k2p = k2 == 0 ? 0 : N - k2;
            const int s_a = ((k2 % R) / P) * 64 + k2 / R;
            const int s_b = ((k2p % R) / P) * 64 + k2p / R;
            cx<T> x[R];
#pragma unroll
            for (int a = 0; a < R; ++a) {
                const int n1 = 64 * a + lane;
                x[a] = {T(0), T(0)};
                if (a < NA && n1 < NK) {
                    const int r = n1 >> 1;
                    const cx<T> z1 = A[r * PITCH + s_a], z2 = conjg(A[r * PITCH + s_b]);
                    // the row pair's spectrum Z = F(2r) + i F(2r+1), times 2
                    x[a] = (n1 & 1) ? times_mi(z1 - z2) : z1 + z2;
                }
            }
            fwd_inlane(x, tw.nat);
            const T s2 = S2[k2];
            // W / 2 (the 2 of the unpacking), the 1/N^2 already in the tables
            auto apply_w = [&](cx<T>& v, int kk) {
                const int dk = kk - k2;
                const T wgt = S1[kk] + s2 + KK[dk < 0 ? dk + N : dk];
                v = times_mi(v);
                v = {v.r * wgt, v.i * wgt};
            };
            if constexpr (TRX) {
                dif64_to_trx<false>(x, tw);
                // slot k: output index br(position), position bits 4, 5 = k >> 1,
                // k & 1 (bits 1, 0 after the reversal); k1 from lane bits 5, 4
                const int k1l = ((lane >> 5) & 1) | (((lane >> 4) & 1) << 1);
                const int brl = (int)(__builtin_bitreverse32((unsigned)(lane & 15)) >> 26);
#pragma unroll
                for (int k = 0; k < 4; ++k) apply_w(x[k], k1l + R * (brl | ((k >> 1) << 1) | (k & 1)));
                dit64_from_trx<true>(x, tw);
            } else {
                dif64<false, SW>(x, tw);
#pragma unroll
                for (int k1 = 0; k1 < R; ++k1) apply_w(x[k1], k1 + R * blane);
                dit64<true, SW>(x, tw);
            }
            inv_inlane(x, tw.nat);
#pragma unroll
            for (int a = 0; a < NA; ++a) {
                const int n1 = 64 * a + lane;
                const cx<T> o = xchg_cx(x[a], 0);  // C(n1 ^ 1, k2)
                if (n1 < NK) {
                    const int r = n1 >> 1;
                    if (!(n1 & 1))
                        A[r * PITCH + s_a] = x[a] + times_i(o);
                    else if (k2p != k2)
                        A[r * PITCH + s_b] = conjg(o) + times_i(conjg(x[a]));
                }
            }
        }
        __syncthreads();

        // inverse row transforms of this pass's frequencies into the registers
        // (unrolled: acc is indexed by q)
#pragma unroll
        for (int q = 0; q < RPW; ++q) {
            const int r = wave * RPW + q;
            cx<T> z[R];
#pragma unroll
            for (int k = 0; k < R; ++k) z[k] = {T(0), T(0)};
            if constexpr (TRX) {
                // read in the transposed layout (see the forward rows)
                const int k1l = ((lane >> 5) & 1) | (((lane >> 4) & 1) << 1);
                if (k1l % P == p) {
                    const int jj = k1l / P;
#pragma unroll
                    for (int k = 0; k < 4; ++k)
                        z[k] = A[r * PITCH + jj * 64 + ((lane & 15) | ((k >> 1) << 4) | ((k & 1) << 5))];
                }
                dif64_from_trx<true>(z, tw);
            } else {
#pragma unroll
                for (int jj = 0; jj < NJ; ++jj) z[p + P * jj] = A[r * PITCH + jj * 64 + lane];
                dif64<true, SW>(z, tw);
            }
            inv_inlane(z, tw.rev);
#pragma unroll
            for (int a = 0; a < NA; ++a) acc[q][a] = acc[q][a] + z[a];
            // one transform at a time: interleaving them spills the accumulators
            __builtin_amdgcn_sched_barrier(0);
        }
        if (p + 1 < P) __syncthreads();
    }

    // rows 2r (real part) and 2r + 1 (imaginary part) at n2 = 64a + br(L)
#pragma unroll
    for (int q = 0; q < RPW; ++q) {
        const int r = wave * RPW + q;
#pragma unroll
        for (int a = 0; a < NA; ++a) {
            const int n2 = 64 * a + blane;
            if (n2 >= NK) continue;
            const long i0 = pbase + (long)(2 * r) * NK + n2;
            T e = alpha * acc[q][a].r, o = alpha * acc[q][a].i;
            if (add_base) {
                e += cu * u[i0];
                o += cu * u[i0 + NK];
                if (v) {
                    e += cv * v[i0];
                    o += cv * v[i0 + NK];
                }
            }
            out[i0] = e;
            out[i0 + NK] = o;
        }
    }
}

template <typename T, int NK>
hipError_t go_fft(const ThetaArgs& a, const T* u, const T* v, T* out, int mode, double tau, hipStream_t st)
{
    using S = FftShape<T, NK>;
    auto kf = k_theta_fft<T, NK>;
    const size_t lds = S::lds();
    hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    const T beta = mode == 1 ? (T)tau : T(0);
    const T alpha = mode == 1 ? (T)(0.5 * tau) : T(1);
    const T cu = mode == 1 ? T(1) : T(0);
    const T cv = mode == 1 ? (T)(0.5 * tau) : T(0);
    hipLaunchKernelGGL(kf, dim3((unsigned)((long)a.nx * a.nx)), dim3(S::NW * 64), lds, st, a.nx, a.fft_sym, u,
                       mode == 1 ? v : nullptr, out, beta, alpha, cu, cv);
    return hipGetLastError();
}

}  // namespace

bool theta_fft_ok(const ThetaArgs& a)
{
    return a.ksem == nullptr &&
           (a.nk == 16 || a.nk == 32 || a.nk == 48 || a.nk == 64 || a.nk == 96 || a.nk == 128) &&
           a.precision != WIG2_BF16X2;
}

template <typename T>
hipError_t launch_theta_fft(const ThetaArgs& a, const T* u, const T* v, T* out, int mode, double tau,
                            hipStream_t st)
{
    if (!theta_fft_ok(a) || a.fft_sym == nullptr || (mode == 1 && v == nullptr)) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_fft_symbols, dim3(a.nx, 3), dim3(256), 0, st, a.nx, a.nk, a.sig1, a.sig2, a.kap,
                       a.fft_sym);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    switch (a.nk) {
    case 16: return go_fft<T, 16>(a, u, v, out, mode, tau, st);
    case 32: return go_fft<T, 32>(a, u, v, out, mode, tau, st);
    case 48: return go_fft<T, 48>(a, u, v, out, mode, tau, st);
    case 64: return go_fft<T, 64>(a, u, v, out, mode, tau, st);
    case 96: return go_fft<T, 96>(a, u, v, out, mode, tau, st);
    default: return go_fft<T, 128>(a, u, v, out, mode, tau, st);
    }
}
template hipError_t launch_theta_fft<double>(const ThetaArgs&, const double*, const double*, double*, int, double,
                                             hipStream_t);
template hipError_t launch_theta_fft<float>(const ThetaArgs&, const float*, const float*, float*, int, double,
                                            hipStream_t);

}  // namespace wig2
