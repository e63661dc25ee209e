// Cubic B-spline advection sweeps (Sec. 4.1) for gfx950.
//
// One lane owns one 1-D line along x_dim at fixed (other x, n1, n2).  Lanes of
// a wavefront take consecutive n2, so every load/store of a wavefront is one
// contiguous 64-element run (coalesced), whichever dimension is swept.  The
// register-resident sweep streams each element through once: its loads and
// stores carry the non-temporal hint.
//
// Spline coefficients: periodic lines solve the circulant system
// (eta_{i-1} + 4 eta_i + eta_{i+1})/6 = g_i exactly by the factorised
// recursive filter 6/(z + 4 + 1/z) = -6 z1 / ((1 - z1/z)(1 - z1 z)),
// z1 = sqrt(3) - 2, with the periodic initial values summed over the whole
// period.  Box lines use the natural end conditions with zero ghost values
// (A_nat of Sec. 4.1), which fix eta_0 = g_0, eta_{n-1} = g_{n-1} and leave a
// (1,4,1) tridiagonal system for the interior (Thomas, multipliers from a
// table).  The displacement c = s p / (m dx) is the same for the whole line,
// so the evaluation at the feet x_i - c dx is a short FIR over the
// coefficients with per-lane taps.
#include "common.h"

#include <cmath>

namespace wig2 {
namespace {

__device__ inline void cubic_weights(double t, double (&w)[4])
{
    const double s = 1.0 - t;
    const double t2 = t * t, t3 = t2 * t;
    w[0] = s * s * s * (1.0 / 6.0);
    w[1] = (3.0 * t3 - 6.0 * t2 + 4.0) * (1.0 / 6.0);
    w[2] = (-3.0 * t3 + 3.0 * t2 + 3.0 * t + 1.0) * (1.0 / 6.0);
    w[3] = t3 * (1.0 / 6.0);
}

// Pole of the periodic spline prefilter, as the element type holds it, and
// the periodic gain 1 / (1 - z1^n) of its start values.
template <typename T>
__host__ __device__ constexpr T spline_pole()
{
    return T(-2.0 + 1.7320508075688772935274463415059);
}
__host__ __device__ constexpr double periodic_gain(double z, int n)
{
    double p = 1.0;
    for (int k = 0; k < n; ++k) p *= z;
    return 1.0 / (1.0 - p);
}

// Evaluation taps of one line, out_i = sum_k a_k eta_{i+J+k-1}, from the
// cubic B-spline weights at t = -c - J, J = floor(-c), times the prefilter
// scale, in FP64.  The scale (1 - z1)^2 for the periodic prefilter of pole z1
// (as held in the element type) makes the DC gain of the whole sweep one for
// that pole (for the exact pole it equals -6 z1).  The tap sum is evaluated
// in FP64 for FP32 lines too and rounded once at the store: accumulated in
// float, it shifts the mass of smooth positive lines by a few 1e-9 per sweep,
// coherently, sweep after sweep.
struct Taps {
    double a[4];
    int J;
};

template <typename T, bool PER>
__device__ inline Taps line_taps(double c)
{
    Taps tp;
    const double mc = -c;
    const double Jd = floor(mc);
    tp.J = (int)Jd;
    double w[4];
    cubic_weights(mc - Jd, w);
    double scale = 1.0;
    if constexpr (PER) {
        const double z1 = (double)spline_pole<T>();
        scale = (1.0 - z1) * (1.0 - z1);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) tp.a[k] = w[k] * scale;
    return tp;
}

// Periodic start value of a first-order recursive filter of pole z over a
// whole period, sum_{k<n} z^k g[(start - dir k) mod n] / (1 - z^n), in FP64
// by Horner's rule.
template <typename T, typename G>
__device__ inline T periodic_start(G g, int n, int start, int dir)
{
    const double z = (double)spline_pole<T>();
    auto at = [&](int k) {
        int j = (start - dir * k) % n;
        return (double)g(j < 0 ? j + n : j);
    };
    double s = at(n - 1);
    for (int k = n - 2; k >= 0; --k) s = s * z + at(k);
    return T(s * periodic_gain(z, n));
}

struct LineMap {
    long base, stride;
    int nv;
};

__device__ inline LineMap line_map(long line, int nx, int nk, int dim)
{
    const long nk2 = (long)nk * nk;
    const long o = line / nk2, rem = line - o * nk2;
    LineMap m;
    if (dim == 1) {  // line along i1 at fixed (i2 = o, n1, n2)
        m.base = o * nk2 + rem;
        m.stride = (long)nx * nk2;
        m.nv = (int)(rem / nk);
    } else {  // line along i2 at fixed (i1 = o, n1, n2)
        m.base = o * nx * nk2 + rem;
        m.stride = nk2;
        m.nv = (int)(rem % nk);
    }
    return m;
}

// ---------------------------------------------------------------------------
// Register-resident line (NX compile-time): loads, solve and FIR unrolled.
// Handles displacements |c| <= 1 cell (taps d in [-2, 2]).
// ---------------------------------------------------------------------------
// PASSES = 2 applies the same sweep twice to the register-resident line
// (two consecutive half-step sweeps along one dimension): the arithmetic of
// each pass, and the rounding of the intermediate line to T, are those of two
// separate launches, without the intermediate round trip through HBM.
template <typename T, int NX, bool PER, int PASSES = 1>
__device__ __forceinline__ void advect_line_core(const T* __restrict__ in, long ib, long is,
                                                 T* __restrict__ out, long ob, long os, double c,
                                                 const double* __restrict__ thomas)
{
    T v[NX];
#pragma unroll
    for (int i = 0; i < NX; ++i) v[i] = __builtin_nontemporal_load(&in[ib + (long)i * is]);

    // c as one rounded value: the taps and the box mask both start from it
    // (no contraction of its product into later arithmetic), so every pass
    // and every launch derives the same taps from it
    asm volatile("" : "+v"(c));
    const Taps tp = line_taps<T, PER>(c);
    // the same taps on the 5-point window d in [-2, 2] around i (|c| <= 1:
    // J in {-1, 0, 1}, and the weight that would fall at d = 3 is zero)
    double ad[5];
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
        const int k = d - tp.J + 1;
        ad[d + 2] = (k == 0) ? tp.a[0] : (k == 1) ? tp.a[1] : (k == 2) ? tp.a[2] : (k == 3) ? tp.a[3] : 0.0;
    }

#pragma unroll
    for (int pass = 0; pass < PASSES; ++pass) {
        T em1 = T(0), eN = T(0);  // box: eta_{-1}, eta_{NX}
        if constexpr (PER) {
            constexpr T z1 = spline_pole<T>();
            constexpr double z1d = (double)z1;
            constexpr double inv = periodic_gain(z1d, NX);
            // Periodic start values, sum_k z1^k g[j_k] / (1 - z1^NX), in FP64
            // by Horner's rule.  FP64 lines sum the whole period; FP32 lines
            // stop after KS terms, where |z1|^KS < 2e-14 of the first term
            // (far below a float's rounding: the sum is exact in FP32).
            constexpr int KS = sizeof(T) == 4 && NX > 24 ? 24 : NX;
            // causal filter: j_k = -k mod NX
            double s = (double)v[(NX - (KS - 1)) % NX];
#pragma unroll
            for (int k = KS - 2; k >= 0; --k) s = s * z1d + (double)v[(NX - k) % NX];
            v[0] = T(s * inv);
#pragma unroll
            for (int i = 1; i < NX; ++i) v[i] += z1 * v[i - 1];
            // anti-causal filter: j_k = NX - 1 + k mod NX
            s = (double)v[(NX - 1 + KS - 1) % NX];
#pragma unroll
            for (int k = KS - 2; k >= 0; --k) s = s * z1d + (double)v[(NX - 1 + k) % NX];
            v[NX - 1] = T(s * inv);
#pragma unroll
            for (int i = NX - 2; i >= 0; --i) v[i] += z1 * v[i + 1];
            // eta = (1 - z1)^2 v; the factor sits in the taps
        } else {
            // natural ends: eta_0 = g_0, eta_{N-1} = g_{N-1}; interior Thomas
            const T e0 = v[0], eL = v[NX - 1];
            T dprev = T(0);
#pragma unroll
            for (int i = 1; i <= NX - 2; ++i) {
                T rhs = T(6) * v[i] - dprev;
                if (i == 1) rhs -= e0;
                if (i == NX - 2) rhs -= eL;
                dprev = rhs * T(thomas[i]);
                v[i] = dprev;
            }
#pragma unroll
            for (int i = NX - 3; i >= 1; --i) v[i] -= T(thomas[i]) * v[i + 1];
            em1 = T(2) * v[0] - v[1];
            eN = T(2) * v[NX - 1] - v[NX - 2];
        }

        T r[NX];  // the line after a pass that is not the last (unused when PASSES = 1)
#pragma unroll
        for (int i = 0; i < NX; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int d = -2; d <= 2; ++d) {
                T e;
                if constexpr (PER) {
                    e = v[(i + d + NX) % NX];
                } else {
                    const int j = i + d;
                    e = (j >= 0 && j < NX) ? v[j < 0 ? 0 : (j >= NX ? NX - 1 : j)]
                                           : (j == -1 ? em1 : (j == NX ? eN : T(0)));
                }
                acc += ad[d + 2] * (double)e;
            }
            T o = T(acc);
            if constexpr (!PER) {
                const double u = (double)i - c;
                if (u < 0.0 || u > (double)(NX - 1)) o = T(0);
            }
            if (pass + 1 < PASSES)
                r[i] = o;
            else
                __builtin_nontemporal_store(o, &out[ob + (long)i * os]);
        }
        if (pass + 1 < PASSES) {
            // the next pass takes the line as opaque values, as a separate
            // launch takes it from memory: no algebra across the passes
#pragma unroll
            for (int i = 0; i < NX; ++i) {
                v[i] = r[i];
                asm volatile("" : "+v"(v[i]));
            }
        }
    }
}

template <typename T, int NX, bool PER, int PASSES = 1>
__device__ __forceinline__ void advect_line_reg(const T* __restrict__ in, T* __restrict__ out,
                                                int nk, int dim, long line, double cpp,
                                                const double* __restrict__ pn,
                                                const double* __restrict__ thomas)
{
    const LineMap lm = line_map(line, NX, nk, dim);
    advect_line_core<T, NX, PER, PASSES>(in, lm.base, lm.stride, out, lm.base, lm.stride,
                                         cpp * pn[lm.nv], thomas);
}

template <typename T, int NX, bool PER, int PASSES>
__global__ __launch_bounds__(64) void k_advect_reg(const T* __restrict__ in, T* __restrict__ out,
                                                   int nk, int dim, long nlines, double cpp,
                                                   const double* __restrict__ pn,
                                                   const double* __restrict__ thomas)
{
    const long line = (long)blockIdx.x * 64 + threadIdx.x;
    if (line >= nlines) return;
    advect_line_reg<T, NX, PER, PASSES>(in, out, nk, dim, line, cpp, pn, thomas);
}

// ---------------------------------------------------------------------------
// Segmented periodic line (NX = NSEG x 32, displacement of at most one cell):
// a workgroup of NSEG waves takes 64 lines, wave s holding segment s (32
// points) of each line in registers, so loads and stores stay one
// contiguous run per wave as in the register-resident sweep.  Each recursive
// filter runs inside the segment from a zero start and is completed with the
// neighbour segment's zero-start end value: the causal value entering
// segment s, sum_{k>=0} z1^k g[start - 1 - k], equals the previous segment's
// zero-start end value up to z1^32 (5e-19) of its size, and likewise for the
// anti-causal filter, so the result is the periodic solve's.  The FIR window
// (two points on each side) takes the neighbours' edge coefficients through
// LDS.  PASSES = 2 applies the sweep twice, as the register-resident kernel.
// ---------------------------------------------------------------------------
template <typename T, int NX, int PASSES>
__global__ __launch_bounds__(NX / 32 * 64) void k_advect_seg(const T* __restrict__ in, T* __restrict__ out,
                                                           int nk, int dim, long nlines, double cpp,
                                                           const double* __restrict__ pn)
{
    constexpr int S = 32, NSEG = NX / S;
    static_assert(NX % S == 0 && NSEG >= 2, "segments of 32 points");
    __shared__ double ends[2][NSEG][64];  // zero-start filter values at the segment ends
    __shared__ T edge[4][NSEG][64];       // first two and last two coefficients
    const int lane = threadIdx.x & 63, sg = threadIdx.x >> 6;
    const int prv = (sg + NSEG - 1) % NSEG, nxt = (sg + 1) % NSEG;
    const long line = (long)blockIdx.x * 64 + lane;
    const bool act = line < nlines;
    const LineMap lm = line_map(act ? line : 0, NX, nk, dim);
    double c = cpp * pn[lm.nv];
    asm volatile("" : "+v"(c));
    const Taps tp = line_taps<T, true>(c);
    double ad[5];
#pragma unroll
    for (int d = -2; d <= 2; ++d) {
        const int k = d - tp.J + 1;
        ad[d + 2] = (k == 0) ? tp.a[0] : (k == 1) ? tp.a[1] : (k == 2) ? tp.a[2] : (k == 3) ? tp.a[3] : 0.0;
    }
    constexpr T z1 = spline_pole<T>();
    constexpr double z1d = (double)z1;
    const long b0 = lm.base + (long)sg * S * lm.stride;
    T v[S];
#pragma unroll
    for (int i = 0; i < S; ++i) v[i] = act ? __builtin_nontemporal_load(&in[b0 + (long)i * lm.stride]) : T(0);

#pragma unroll
    for (int pass = 0; pass < PASSES; ++pass) {
        // causal filter: zero start, then the entering value from segment s-1
#pragma unroll
        for (int i = 1; i < S; ++i) v[i] += z1 * v[i - 1];
        ends[0][sg][lane] = (double)v[S - 1];
        __syncthreads();
        {
            const double t = ends[0][prv][lane];
            double zp = z1d;
#pragma unroll
            for (int i = 0; i < S; ++i) {
                v[i] = T((double)v[i] + zp * t);
                zp *= z1d;
            }
        }
        // anti-causal filter: zero start at the segment end, then the value
        // entering from segment s+1
#pragma unroll
        for (int i = S - 2; i >= 0; --i) v[i] += z1 * v[i + 1];
        ends[1][sg][lane] = (double)v[0];
        __syncthreads();
        {
            const double h = ends[1][nxt][lane];
            double zp = z1d;
#pragma unroll
            for (int i = S - 1; i >= 0; --i) {
                v[i] = T((double)v[i] + zp * h);
                zp *= z1d;
            }
        }
        edge[0][sg][lane] = v[0];
        edge[1][sg][lane] = v[1];
        edge[2][sg][lane] = v[S - 2];
        edge[3][sg][lane] = v[S - 1];
        __syncthreads();
        const T em2 = edge[2][prv][lane], em1 = edge[3][prv][lane];
        const T ep0 = edge[0][nxt][lane], ep1 = edge[1][nxt][lane];
        auto eta = [&](int j) -> T { return j == -2 ? em2 : j == -1 ? em1 : j == S ? ep0 : j == S + 1 ? ep1 : v[j]; };
        T r[S];
#pragma unroll
        for (int i = 0; i < S; ++i) {
            double acc = 0.0;
#pragma unroll
            for (int d = -2; d <= 2; ++d) acc += ad[d + 2] * (double)eta(i + d);
            r[i] = T(acc);
        }
        if (pass + 1 < PASSES) {
#pragma unroll
            for (int i = 0; i < S; ++i) {
                v[i] = r[i];
                asm volatile("" : "+v"(v[i]));
            }
        } else if (act) {
#pragma unroll
            for (int i = 0; i < S; ++i) __builtin_nontemporal_store(r[i], &out[b0 + (long)i * lm.stride]);
        }
    }
}

// ---------------------------------------------------------------------------
// General line (any nx, any displacement): the coefficients go through a
// state-sized scratch array laid out like the state (coalesced).
// ---------------------------------------------------------------------------
template <typename T, bool PER>
__global__ __launch_bounds__(64) void k_advect_any(const T* __restrict__ in, T* __restrict__ out,
                                                   T* __restrict__ ws, int nx, int nk, int dim,
                                                   long nlines, double cpp,
                                                   const double* __restrict__ pn,
                                                   const double* __restrict__ thomas)
{
    const long line = (long)blockIdx.x * 64 + threadIdx.x;
    if (line >= nlines) return;
    const LineMap lm = line_map(line, nx, nk, dim);
    double c = cpp * pn[lm.nv];
    asm volatile("" : "+v"(c));
    auto G = [&](int i) { return in[lm.base + (long)i * lm.stride]; };
    auto E = [&](int i) -> T& { return ws[lm.base + (long)i * lm.stride]; };
    T em1 = T(0), eN = T(0);
    if constexpr (PER) {
        const T z1 = spline_pole<T>();
        T prev = periodic_start<T>(G, nx, 0, 1);
        E(0) = prev;
        for (int i = 1; i < nx; ++i) {
            prev = G(i) + z1 * prev;
            E(i) = prev;
        }
        prev = periodic_start<T>([&](int j) { return E(j); }, nx, nx - 1, -1);
        E(nx - 1) = prev;
        for (int i = nx - 2; i >= 0; --i) {
            prev = E(i) + z1 * prev;
            E(i) = prev;
        }
    } else {
        const T e0 = G(0), eL = G(nx - 1);
        E(0) = e0;
        E(nx - 1) = eL;
        T dprev = T(0);
        for (int i = 1; i <= nx - 2; ++i) {
            T rhs = T(6) * G(i) - dprev;
            if (i == 1) rhs -= e0;
            if (i == nx - 2) rhs -= eL;
            dprev = rhs * T(thomas[i]);
            E(i) = dprev;
        }
        for (int i = nx - 3; i >= 1; --i) E(i) = E(i) - T(thomas[i]) * E(i + 1);
        em1 = T(2) * E(0) - E(1);
        eN = T(2) * E(nx - 1) - E(nx - 2);
    }
    const Taps tp = line_taps<T, PER>(c);
    const long J = tp.J;
    for (int i = 0; i < nx; ++i) {
        double acc = 0.0;
        if (PER || ((double)i - c >= 0.0 && (double)i - c <= (double)(nx - 1))) {
            for (int k = 0; k < 4; ++k) {
                long j = (long)i + J + k - 1;
                T e;
                if constexpr (PER) {
                    j %= nx;
                    if (j < 0) j += nx;
                    e = E((int)j);
                } else {
                    e = (j >= 0 && j < nx) ? E((int)j) : (j == -1 ? em1 : (j == nx ? eN : T(0)));
                }
                acc += tp.a[k] * (double)e;
            }
        }
        out[lm.base + (long)i * lm.stride] = T(acc);
    }
}


// ---------------------------------------------------------------------------
// Batched sweep: every wave takes 64-line items from a list spanning all
// instances of an ensemble (grid-stride, items pre-sorted by cost).
// ---------------------------------------------------------------------------
template <typename T, int NX, int PASSES>
__global__ __launch_bounds__(256) void k_advect_batch(const T* __restrict__ in_pool,
                                                      T* __restrict__ out_pool,
                                                      const BatchInst* __restrict__ insts,
                                                      const AdvItem* __restrict__ items, int nitems,
                                                      int dim, const double* __restrict__ p_pool)
{
    const int lane = threadIdx.x & 63;
    const int nwaves = gridDim.x * 4;
    for (int it = (blockIdx.x * 256 + threadIdx.x) >> 6; it < nitems; it += nwaves) {
        const AdvItem item = items[it];
        const BatchInst I = insts[item.inst];
        const long line = item.line0 + lane;
        if (line >= (long)NX * I.nk * I.nk) continue;
        advect_line_reg<T, NX, true, PASSES>(in_pool + I.off, out_pool + I.off, I.nk, dim, line, I.cpp,
                                             p_pool + I.p_off, nullptr);
    }
}

template <typename T, int NX, bool PER>
hipError_t run_reg(const T* in, T* out, int nk, int dim, long nl, double cpp, const double* p,
                   const double* th, int passes, hipStream_t st)
{
    const unsigned nb = (unsigned)((nl + 63) / 64);
    if (passes == 2)
        hipLaunchKernelGGL((k_advect_reg<T, NX, PER, 2>), dim3(nb), dim3(64), 0, st, in, out, nk,
                           dim, nl, cpp, p, th);
    else
        hipLaunchKernelGGL((k_advect_reg<T, NX, PER, 1>), dim3(nb), dim3(64), 0, st, in, out, nk,
                           dim, nl, cpp, p, th);
    return hipGetLastError();
}

}  // namespace

bool batch_nx_ok(int nx)
{
    return nx == 16 || nx == 32 || nx == 48 || nx == 64 || nx == 96 || nx == 128;
}

template <typename T>
hipError_t launch_advect_batch(const T* in_pool, T* out_pool, const BatchInst* insts,
                               const AdvItem* items, int nitems, int dim, const double* p_pool,
                               int nx, int grid, hipStream_t st, int passes)
{
    if (nitems == 0) return hipSuccess;
    if (passes != 1 && passes != 2) return hipErrorInvalidValue;
#define WIG2_ADV_BATCH(N)                                                                          \
    case N:                                                                                        \
        if (passes == 2)                                                                           \
            hipLaunchKernelGGL((k_advect_batch<T, N, 2>), dim3(grid), dim3(256), 0, st, in_pool,    \
                               out_pool, insts, items, nitems, dim, p_pool);                       \
        else                                                                                       \
            hipLaunchKernelGGL((k_advect_batch<T, N, 1>), dim3(grid), dim3(256), 0, st, in_pool,    \
                               out_pool, insts, items, nitems, dim, p_pool);                       \
        return hipGetLastError();
    switch (nx) {
        WIG2_ADV_BATCH(16)
        WIG2_ADV_BATCH(32)
        WIG2_ADV_BATCH(48)
        WIG2_ADV_BATCH(64)
        WIG2_ADV_BATCH(96)
        WIG2_ADV_BATCH(128)
    default: return hipErrorInvalidValue;
    }
#undef WIG2_ADV_BATCH
}
template hipError_t launch_advect_batch<double>(const double*, double*, const BatchInst*,
                                                const AdvItem*, int, int, const double*, int, int,
                                                hipStream_t, int);
template hipError_t launch_advect_batch<float>(const float*, float*, const BatchInst*,
                                               const AdvItem*, int, int, const double*, int, int,
                                               hipStream_t, int);

bool advect_in_registers(int nx, bool periodic, double max_cells)
{
    if (!(max_cells <= 1.0)) return false;
    if (periodic) return nx == 16 || nx == 32 || nx == 48 || nx == 64 || nx == 96 || nx == 128 || nx == 256;
    return nx == 33 || nx == 65 || nx == 129;
}

template <typename T>
hipError_t launch_advect(const T* in, T* out, T* work, int nx, int nk, int dim, bool periodic,
                         double cpp, double max_cells, const double* p_dev,
                         const double* thomas_dev, hipStream_t st, int passes)
{
    const long nl = (long)nx * nk * nk;
    if (nl == 0) return hipSuccess;
    if (passes != 1 && !(passes == 2 && advect_in_registers(nx, periodic, max_cells)))
        return hipErrorInvalidValue;
    if (advect_in_registers(nx, periodic, max_cells)) {
        if (periodic) {
            switch (nx) {
            case 16: return run_reg<T, 16, true>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            case 32: return run_reg<T, 32, true>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            case 48: return run_reg<T, 48, true>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            case 64: return run_reg<T, 64, true>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            case 96: return run_reg<T, 96, true>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            case 128: return run_reg<T, 128, true>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            case 256: {
                const unsigned nb = (unsigned)((nl + 63) / 64);
                if (passes == 2)
                    hipLaunchKernelGGL((k_advect_seg<T, 256, 2>), dim3(nb), dim3(512), 0, st, in, out, nk, dim, nl,
                                       cpp, p_dev);
                else
                    hipLaunchKernelGGL((k_advect_seg<T, 256, 1>), dim3(nb), dim3(512), 0, st, in, out, nk, dim, nl,
                                       cpp, p_dev);
                return hipGetLastError();
            }
            default: break;
            }
        } else {
            switch (nx) {
            case 33: return run_reg<T, 33, false>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            case 65: return run_reg<T, 65, false>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            case 129: return run_reg<T, 129, false>(in, out, nk, dim, nl, cpp, p_dev, thomas_dev, passes, st);
            default: break;
            }
        }
    }
    if (!work) return hipErrorInvalidValue;
    const unsigned nb = (unsigned)((nl + 63) / 64);
    if (periodic)
        hipLaunchKernelGGL((k_advect_any<T, true>), dim3(nb), dim3(64), 0, st, in, out, work, nx,
                           nk, dim, nl, cpp, p_dev, thomas_dev);
    else
        hipLaunchKernelGGL((k_advect_any<T, false>), dim3(nb), dim3(64), 0, st, in, out, work, nx,
                           nk, dim, nl, cpp, p_dev, thomas_dev);
    return hipGetLastError();
}

template hipError_t launch_advect<double>(const double*, double*, double*, int, int, int, bool,
                                          double, double, const double*, const double*,
                                          hipStream_t, int);
template hipError_t launch_advect<float>(const float*, float*, float*, int, int, int, bool, double,
                                         double, const double*, const double*, hipStream_t, int);

}  // namespace wig2
