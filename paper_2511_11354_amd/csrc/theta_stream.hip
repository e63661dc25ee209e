// Streaming Theta kernel for the torus when the single-body symbols have a
// narrow band (a few Fourier modes of V_ext, Sec. 3.1.1): the pair term
// (Sec. 3.1.2, eq. two_body_FSM) is the only dense contraction and runs on
// the matrix cores; the single-body differences run on the vector ALUs.
//
// One workgroup of NK/16 waves is resident per slot and walks the planes
// p = blockIdx.x, blockIdx.x + gridDim.x, ...  While the matrix cores work on
// plane p from LDS, the global loads of plane p + gridDim.x are in flight
// into registers; they are written to LDS once every wave is done with p.
// The pair-term accumulators are in skewed coordinates (n1, s = n1 + n2) and
// every valid accumulator element is exactly one plane point, so each lane
// finishes its points in place (single-body terms from LDS, epilogue, store)
// without the scatter through LDS the general kernel needs.
//
// Epilogue forms (x: the plane the operator acts on, y: a second state):
//   form 0: out = Theta[x]
//   form 1: out = x + tau Theta[x]
//   form 2: out = (y + x)/2 + (tau/2) Theta[x]
//   form 3: out = x + (tau/2)(Theta[x] + Theta[x + tau Theta[x]]), the whole
//           Heun step with the plane kept in LDS between the two passes
//           (Theta acts within each x-pair plane), so f is read and the
//           result written once; evaluated as h + Theta[(tau/2) g] with
//           h = x + (tau/2) Theta[x], g = x + tau Theta[x].
// Heun's step f + (tau/2)(Theta f + Theta g), g = f + tau Theta f, is form 1
// followed by form 2 with x = g, y = f, because (tau/2) Theta f = (g - f)/2.
// out may alias x or y: plane p of x is read (into registers) one iteration
// before plane p of out is written, and y is read by the lane that writes
// the same element.
#include "common.h"
#include "mfma.h"

#include <algorithm>

namespace wig2 {
namespace {
using namespace mf;


template <typename T>
struct Vec16;
template <>
struct Vec16<double> {
    typedef double V __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};
template <>
struct Vec16<float> {
    typedef float V __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};

// LDS plane: rows -PADR .. NK+PADR-1 at pitch LD = NK + PADC; the PADR
// rows above and below the plane and the PADC columns after each row stay
// zero, so every read of the single-body differences (rows n1 +- m, columns
// n2 +- m, m <= kStreamBand) and of the skewed pair operand of a visited
// tile (columns -15 .. NK+15: a column c < 0 of row k is column LD + c of
// row k - 1) lands on plane data or on a zero, with no bounds test.  PADC
// >= 16 is chosen with LD - 1 = 16 (mod 32): the four k-rows of an operand
// read (row step LD - 1 in the skewed layout) then fall on disjoint groups
// of LDS banks, for 4- and 8-byte elements.
template <typename T, int NK>
struct StreamLayout {
    static constexpr int PADR = kStreamBand;
    static constexpr int R32 = ((17 - NK) % 32 + 32) % 32;  // LD - 1 = 16 (mod 32)
    static constexpr int PADC = R32 >= 16 ? R32 : R32 + 32;
    static constexpr int LD = NK + PADC;
    static constexpr int X_ELEMS = (NK + 2 * PADR) * LD;
    static constexpr int TAB = 2 * NK;
    static constexpr size_t bytes = sizeof(T) * (size_t)(X_ELEMS + TAB);
};

// Waves per SIMD to budget registers for: FP32 planes of 128 fit twice in
// LDS, so two 8-wave workgroups share a CU when a wave stays within 128 VGPRs
// (the one-pass Heun form then drops its register prefetch of the next plane:
// the other workgroup's matrix-core work covers the loads; 4% faster than one
// workgroup with the prefetch, bitwise the same).
template <typename T, int NK, int FORM, int WS>
constexpr int stream_waves_per_eu()
{
    return (sizeof(T) == 4 && NK == 128 && WS == 1) ? 4 : (sizeof(T) == 4 && NK <= 64) ? 2 : 1;
}
// The batched kernel loads each plane at the top of its loop.
template <typename T, int NK>
constexpr int batch_stream_waves_per_eu()
{
    return (sizeof(T) == 4 && NK <= 64) ? 2 : 1;
}

// Theta work on one plane held in LDS (X, and tk for the pair term), after
// the barrier that published it: both passes for the one-pass Heun form,
// one pass and the epilogue otherwise.  Ends with a barrier, after which X
// may be rewritten.  Every thread of the workgroup calls it.  The one-pass
// Heun form calls before_pass2() once the first pass no longer reads the
// plane's registers (the caller issues the next plane's loads there).
struct NoHook {
    __device__ void operator()() const {}
};
template <typename T, int NK, bool TWO, int FORM, int WS, typename Hook = NoHook>
__device__ __forceinline__ void stream_plane(const T* y, T* out, int nx, long pl, const double* __restrict__ sig1,
                                             const double* __restrict__ sig2, int band, double tau, T* X,
                                             const T* tk, int lane, int w, int J0, Hook before_pass2 = Hook())
{
    typedef typename Acc<T>::V V;
    typedef StreamLayout<T, NK> L;
    constexpr int NW = NK / 16;
    constexpr int NS = NW + 1;
    constexpr int NSH = (NS + WS - 1) / WS;
    constexpr int LD = L::LD;
    const int li = lane & 15, lk = lane >> 4;

    const int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
    const long pbase = pl * (long)NK * NK;

    // Lane-owned points: accumulator element (jj, q) is the point
    // n1 = 16w + acc_row(lk, q), n2 = 16(w + j) + li - n1 of skewed tile
    // j = J0 + jj, when j < NS and 0 <= n2 < NK.
    // Reads for points outside the plane hit the zero gaps (or clamp) and
    // their results are not stored.
    // Position arithmetic restarts from an opaque copy of the lane id in
    // each loop body, so the compiler cannot hoist the 4*NS per-point
    // addresses and masks out of the loops and keep them all live.
    auto opaque_lane = [&]() {
        int l = lane;
        asm volatile("" : "+v"(l));
        return l;
    };
    int el = opaque_lane();
    auto col = [&](int jj, int q) {
        return 16 * (w + J0 + jj) + (el & 15) - (16 * w + acc_row<T>(el >> 4, q));
    };
    auto tile_ok = [&](int jj) { return WS == 1 || J0 + jj < NS; };  // wave-uniform
    auto row = [&](int q) { return 16 * w + acc_row<T>(el >> 4, q); };
    auto lds_at = [&](int j, int q) { return X + row(q) * LD + col(j, q); };

    // acc (+)= Theta of the plane held in X, at the lane-owned points
    auto theta_pass = [&](V (&acc)[NSH], bool accumulate) {
        if (!accumulate) {
#pragma unroll
            for (int j = 0; j < NSH; ++j) acc[j] = V{0, 0, 0, 0};
        }
        if constexpr (TWO) {
            // Output tile (row block w, skewed tile j) covers s in
            // [16(w+j), 16(w+j)+16); the 16 rows k of block KB hold non-zero
            // H[k][s] = X[k][s - k] for that tile iff 0 <= w + j - KB <= NW.
            // A = tk[r - k + NK] (r = 16w + li), B = X[k LD + s - k] (zero gaps
            // outside the plane).
            const T* pa = tk + 16 * w + li + NK - lk;
            const T* pb = X + lk * (LD - 1) + 16 * (w + J0) + li;
            // Operands of k-step kb + 1 are read from LDS while the matrix
            // cores work on k-step kb (two register sets, software
            // pipelined).  All operand reads are issued regardless of the
            // (scalar) tile tests; reads of inactive tiles stay inside the
            // LDS allocation (columns -127 .. 255 of rows 0 .. NK-1) and are
            // not used.
            // Tiles outside the band of wave w: skipped by a wave-uniform
            // branch, or (kZeroA) multiplied with a zero A operand.  At the
            // smaller planes the compiler turns the skip branches into
            // copies of the whole accumulator set at every join (thousands
            // of moves, and spills at FP32 nk = 96), which costs more than
            // the extra products (a wave then issues all (NW + 1) NW tile
            // steps instead of (2 NW + 1) / (3 NW) of them, 72-83% here);
            // the operands of a skipped tile are finite LDS values (plane,
            // zero gaps, kernel table), so 0 * B adds an exact zero.
            constexpr bool kZeroA = sizeof(T) == 4 ? NK < 128 : NK < 64;
            // FP64 planes of 96 and 128: loop over the k-block offset
            // d = KB - w instead.  The A operand depends on d alone, and the
            // tiles j that meet k-block KB = w + d are j in
            // [max(0, d), min(NW, d + NW)], fixed per d, so one wave-uniform
            // test per k-block (is w + d a k-block) replaces the per-tile
            // tests.  Same products in the same order per tile (KB
            // ascending): bitwise the per-tile form, 3-6% faster; FP32 at 128
            // measured 1.5% slower with it and keeps the per-tile form.
            constexpr bool kBlockOffset = !kZeroA && WS == 1 && sizeof(T) == 8 && NK >= 96;
            if constexpr (kBlockOffset) {
                const T* pa0 = tk + li + NK - lk;
                const T* pb0 = X + lk * (LD - 1) + 16 * w * LD + li;
                T a[2], bv[2][NSH];
#pragma unroll
                for (int d = -(NW - 1); d <= NW - 1; ++d) {
                    if (w + d < 0 || w + d >= NW) continue;  // wave-uniform
                    const int lo = d < 0 ? 0 : d, hi = d < 0 ? d + NW : NW;
                    auto load = [&](int i, int buf) {
                        a[buf] = pa0[-16 * d - 4 * i];
                        const T* pb = pb0 + (16 * d + 4 * i) * (LD - 1);
#pragma unroll
                        for (int j = 0; j < NSH; ++j)
                            if (j >= lo && j <= hi) bv[buf][j] = pb[16 * j];
                    };
                    load(0, 0);
#pragma unroll
                    for (int i = 0; i < 4; ++i) {
                        const int cur = i & 1;
                        if (i + 1 < 4) load(i + 1, cur ^ 1);
#pragma unroll
                        for (int j = 0; j < NSH; ++j)
                            if (j >= lo && j <= hi) acc[j] = mma(a[cur], bv[cur][j], acc[j]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
            } else {
            T a[2], bv[2][NSH];
            auto load = [&](int kb, int buf) {
                a[buf] = pa[-4 * kb];
#pragma unroll
                for (int j = 0; j < NSH; ++j) bv[buf][j] = pb[4 * kb * (LD - 1) + 16 * j];
            };
            load(0, 0);
#pragma unroll
            for (int KB = 0; KB < NW; ++KB) {
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int kb = 4 * KB + i, cur = kb & 1;
                    if (kb + 1 < 4 * NW) load(kb + 1, cur ^ 1);
#pragma unroll
                    for (int j = 0; j < NSH; ++j) {
                        const int d = w + J0 + j - KB;
                        if (!tile_ok(j)) continue;
                        if constexpr (kZeroA) {
                            const T as = (d < 0 || d > NW) ? T(0) : a[cur];
                            acc[j] = mma(as, bv[cur][j], acc[j]);
                        } else {
                            if (d < 0 || d > NW) continue;  // wave-uniform
                            acc[j] = mma(a[cur], bv[cur][j], acc[j]);
                        }
                    }
                    // keep the scheduler from hoisting further operand
                    // reads of the unrolled loop (register pressure)
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            }
        }
        // single-body differences (modes 1..band of x_i1 along n1, of x_i2
        // along n2), added onto the pair-term accumulators
        for (int m = 1; m <= band; ++m) {
            el = opaque_lane();
            const T s1 = T(sig1[(long)i1 * NK + m]);
            const T s2 = T(sig2[(long)i2 * NK + m]);
            if constexpr (sizeof(T) == 4 && NK < 128) {
                if (m == 1) {
                    // FP32 tiles put a lane's four points on consecutive
                    // rows of one anti-diagonal, (n1 + q, n2 - q), so their
                    // 16 neighbours at distance 1 are 10 distinct values:
                    // rm[t] = f(n1 + t, n2 - t - 1), t = -1..3, and
                    // rp[t] = f(n1 + t, n2 - t + 1), t = 0..4, at fixed
                    // offsets t (LD - 1) -+ 1 from the first point (4-6%
                    // faster launches at nk = 64, 96; at 128, whose one-pass
                    // Heun form runs at 128 VGPRs, the extra live values
                    // spill and it measured 7% slower).
#pragma unroll
                    for (int j = 0; j < NSH; ++j) {
                        const T* b = lds_at(j, 0);
                        T rm[5], rp[5];
#pragma unroll
                        for (int t = 0; t < 5; ++t) {
                            rm[t] = b[(t - 1) * (LD - 1) - 1];
                            rp[t] = b[t * (LD - 1) + 1];
                        }
#pragma unroll
                        for (int q = 0; q < 4; ++q)
                            acc[j][q] += s1 * (rm[q] - rp[q + 1]) + s2 * (rm[q + 1] - rp[q]);
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    continue;
                }
            }
#pragma unroll
            for (int j = 0; j < NSH; ++j) {
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    const T* xp = lds_at(j, q);
                    acc[j][q] += s1 * (xp[-m * LD] - xp[m * LD]) + s2 * (xp[-m] - xp[m]);
                }
                __builtin_amdgcn_sched_barrier(0);
            }
        }
    };

    V sacc[NSH];
    theta_pass(sacc, false);

    if constexpr (FORM == 3) {
        // Whole Heun step in one pass over the plane: h = f + tau/2 Theta f
        // stays in registers and g = f + tau Theta f replaces f in LDS.
        // FP64: LDS holds (tau/2) g instead, and the second pass accumulates
        // Theta[(tau/2) g] = (tau/2) Theta g (Theta is linear) directly onto
        // h (its accumulators are h, so the pass-one results need no
        // registers of their own during pass 2).  FP32 keeps g and h apart
        // and forms h + (tau/2) Theta g at the end: accumulating onto h would
        // round at the scale of h once per matrix-core instruction, which
        // biases the mass measurably over many steps, and the scaled operand
        // adds a rounding to every product.
        constexpr bool ONTO_H = sizeof(T) == 8;
        V hv[NSH];
        el = opaque_lane();
#pragma unroll
        for (int j = 0; j < NSH; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const T fx = *lds_at(j, q);
                hv[j][q] = fx + T(0.5 * tau) * sacc[j][q];
                sacc[j][q] = ONTO_H ? T(0.5 * tau) * (fx + T(tau) * sacc[j][q]) : fx + T(tau) * sacc[j][q];
            }
        __syncthreads();  // every wave is done reading f
        el = opaque_lane();
#pragma unroll
        for (int j = 0; j < NSH; ++j)
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n2 = col(j, q);
                if (tile_ok(j) && n2 >= 0 && n2 < NK) *lds_at(j, q) = sacc[j][q];
            }
        __syncthreads();
        before_pass2();
        if constexpr (ONTO_H) {
            theta_pass(hv, true);
        } else {
            theta_pass(sacc, false);
#pragma unroll
            for (int j = 0; j < NSH; ++j) hv[j] += T(0.5 * tau) * sacc[j];
        }
        el = opaque_lane();
#pragma unroll
        for (int j = 0; j < NSH; ++j) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n1 = row(q), n2 = col(j, q);
                if (tile_ok(j) && n2 >= 0 && n2 < NK) out[pbase + (long)n1 * NK + n2] = hv[j][q];
            }
            __builtin_amdgcn_sched_barrier(0);
        }
        __syncthreads();  // LDS plane is rewritten next
        return;
    }

    // epilogue and store; y (form 2) is fetched one group of tiles ahead
    constexpr int YG = 1;
    constexpr int NG = (NSH + YG - 1) / YG;
    T yv[2][YG][4];
    auto fetch_y = [&](int g, T (&dst)[YG][4]) {
#pragma unroll
        for (int jj = 0; jj < YG; ++jj) {
            const int j = g * YG + jj;
            if (j >= NSH) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n1 = row(q);
                const int c = min(max(col(j, q), 0), NK - 1);
                dst[jj][q] = y[pbase + (long)n1 * NK + c];
            }
        }
    };
    el = opaque_lane();
    if constexpr (FORM == 2) fetch_y(0, yv[0]);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if constexpr (FORM == 2) {
            if (g + 1 < NG) fetch_y(g + 1, yv[(g + 1) & 1]);
        }
#pragma unroll
        for (int jj = 0; jj < YG; ++jj) {
            const int j = g * YG + jj;
            if (j >= NSH) break;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const int n1 = row(q);
                const int n2 = col(j, q);
                const T val = sacc[j][q];
                T o;
                if constexpr (FORM == 0)
                    o = val;
                else if constexpr (FORM == 1)
                    o = *lds_at(j, q) + T(tau) * val;
                else
                    o = T(0.5) * (yv[g & 1][jj][q] + *lds_at(j, q)) + T(0.5 * tau) * val;
                if (tile_ok(j) && n2 >= 0 && n2 < NK) out[pbase + (long)n1 * NK + n2] = o;
            }
        }
        __builtin_amdgcn_sched_barrier(0);
    }
    __syncthreads();  // LDS plane is rewritten next
}

// WS waves share each 16-row block (WS = 2: 2 NK/16 waves per workgroup, each
// with about half of the block's skewed tiles), trading registers per wave
// for more waves to hide LDS and issue latency behind the matrix cores.
template <typename T, int NK, bool TWO, int FORM, int WS>
__global__ __launch_bounds__(NK / 16 * 64 * WS, (stream_waves_per_eu<T, NK, FORM, WS>())) void k_theta_stream(
    const T* x, const T* y, T* out, int nx, long np, const double* __restrict__ sig1,
    const double* __restrict__ sig2, int band, const double* __restrict__ kap, double tau)
{
    typedef typename Acc<T>::V V;
    typedef typename Vec16<T>::V VT;
    typedef StreamLayout<T, NK> L;
    constexpr int NW = NK / 16;
    constexpr int NT = NW * 64 * WS;
    constexpr int NS = NW + 1;                // skewed tiles per row block
    constexpr int NSH = (NS + WS - 1) / WS;   // of which one wave holds
    constexpr int LD = L::LD;
    constexpr int VN = Vec16<T>::N;
    constexpr int NV = NK * NK / (NT * VN);  // 16-byte loads per thread per plane
    static_assert(NK * NK % (NT * VN) == 0, "plane must split into 16-byte loads");

    extern __shared__ unsigned char smem_raw[];
    T* Xbase = reinterpret_cast<T*>(smem_raw);
    T* X = Xbase + L::PADR * LD;  // X[n1 * LD + n2]
    T* tk = Xbase + L::X_ELEMS;   // tk[d + NK] = sgn(d) kap[|d|]

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform (scalar)
    const int w = wv % NW;              // row block
    const int J0 = (wv / NW) * NSH;     // first skewed tile of this wave

    // zero gaps once; plane writes never touch them
    for (int e = tid; e < L::PADR * LD; e += NT) {
        Xbase[e] = T(0);
        X[NK * LD + e] = T(0);
    }
    for (int e = tid; e < NK * L::PADC; e += NT) X[(e / L::PADC) * LD + NK + e % L::PADC] = T(0);

    long pl = blockIdx.x;
    if (pl >= np) return;  // whole workgroup leaves together
    const long stride = gridDim.x;

    // registers of the plane to be written to LDS next.  Nothing consumes
    // them before the next iteration, so the loads stay in flight across the
    // matrix-core work (any arithmetic on a loaded value here would make the
    // wave wait for every load issued before it).
    VT xr[NV];
    double kraw = 0.0;  // kap[l][|d|] of the next plane, d = tid - NK
    // thread id through an opaque copy: per-element addresses are rebuilt
    // per plane instead of being hoisted out of the plane loop and kept live
    auto opaque_tid = [&]() {
        int t = tid;
        asm volatile("" : "+v"(t));
        return t;
    };
    // The one-pass Heun form prefetches the first NVP loads of the next
    // plane during its second pass (at nk = 128 FP64: half of them, the
    // second pass has no room for the whole plane in registers; none for
    // FP32 at 128, which runs two workgroups per CU instead, nor at smaller
    // planes, where the spare registers buy more resident waves) and issues
    // the rest at the top of the next iteration.
    constexpr int NVP = FORM != 3 ? NV : (NK == 128 && sizeof(T) == 8) ? NV / 2 : 0;
    auto fetch_range = [&](long p, int v0, int v1) {
        const VT* src = reinterpret_cast<const VT*>(x + p * (long)NK * NK);
        const int ot = opaque_tid();
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (v >= v0 && v < v1) xr[v] = src[ot + v * NT];
    };
    auto fetch = [&](long p) {
        fetch_range(p, 0, FORM == 3 ? NVP : NV);
        if constexpr (TWO) {
            if (tid < 2 * NK) {
                const int i1 = (int)(p / nx), i2 = (int)(p % nx);
                const int ell = (i1 - i2 + nx) % nx;
                const int d = tid - NK, ad = d < 0 ? -d : d;
                kraw = kap[(long)ell * NK + min(max(ad, 1), NK - 1)];
            }
        }
    };
    // The one-pass Heun form issues the next plane's loads before its
    // second pass, once the first pass's registers are free.
    fetch(pl);

    for (; pl < np; pl += stride) {
        if constexpr (FORM == 3 && NVP < NV) fetch_range(pl, NVP, NV);
        const int ot = opaque_tid();
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int e = (ot + v * NT) * VN;
            *reinterpret_cast<VT*>(X + (e / NK) * LD + e % NK) = xr[v];
        }
        if constexpr (TWO) {
            if (tid < 2 * NK) {
                const int d = tid - NK, ad = d < 0 ? -d : d;
                tk[tid] = (ad > 0 && ad < NK) ? sgnval(d, T(kraw)) : T(0);
            }
        }
        __syncthreads();
        if constexpr (FORM == 3) {
            const long next = pl + stride;
            stream_plane<T, NK, TWO, FORM, WS>(y, out, nx, pl, sig1, sig2, band, tau, X, tk, lane, w, J0,
                                               [&]() {
                                                   if (next < np) fetch(next);
                                               });
        } else {
            if (pl + stride < np) fetch(pl + stride);
            stream_plane<T, NK, TWO, FORM, WS>(y, out, nx, pl, sig1, sig2, band, tau, X, tk, lane, w, J0);
        }
    }
}

// Waves per row block for each plane size and form.
template <typename T, int NK, int FORM>
constexpr int stream_ws()
{
    return 1;
}

template <typename T, int NK, bool TWO, int FORM>
hipError_t go_stream(const ThetaArgs& a, const T* x, const T* y, T* out, double tau, hipStream_t st)
{
    constexpr int WS = stream_ws<T, NK, FORM>();
    auto kf = k_theta_stream<T, NK, TWO, FORM, WS>;
    const size_t sm = StreamLayout<T, NK>::bytes;
    const int nt = NK / 16 * 64 * WS;
    hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    int dev = 0, ncu = 0, per = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, kf, nt, sm)) != hipSuccess) return e;
    const long np = (long)a.nx * a.nx;
    const long grid = std::min<long>(np, (long)std::max(per, 1) * ncu);
    hipLaunchKernelGGL(kf, dim3((unsigned)grid), dim3(nt), sm, st, x, y, out, a.nx, np, a.sig1,
                       a.sig2, a.band, a.kap, tau);
    return hipGetLastError();
}

template <typename T, int NK, bool TWO>
hipError_t go_stream_form(const ThetaArgs& a, const T* x, const T* y, T* out, int form, double tau,
                          hipStream_t st)
{
    switch (form) {
    case 0: return go_stream<T, NK, TWO, 0>(a, x, y, out, tau, st);
    case 1: return go_stream<T, NK, TWO, 1>(a, x, y, out, tau, st);
    case 2: return go_stream<T, NK, TWO, 2>(a, x, y, out, tau, st);
    case 3: return go_stream<T, NK, TWO, 3>(a, x, y, out, tau, st);
    default: return hipErrorInvalidValue;
    }
}

template <typename T, int NK>
hipError_t go_stream_nk(const ThetaArgs& a, const T* x, const T* y, T* out, int form, double tau,
                        hipStream_t st)
{
    return a.kap ? go_stream_form<T, NK, true>(a, x, y, out, form, tau, st)
                 : go_stream_form<T, NK, false>(a, x, y, out, form, tau, st);
}


// ---------------------------------------------------------------------------
// Batched ensembles: one persistent launch per size class walks a list of
// (instance, planes) items and advances each plane by the one-pass Heun form
// in place (the same per-plane arithmetic as a single context).
// ---------------------------------------------------------------------------
template <typename T, int NK>
__global__ __launch_bounds__(NK / 16 * 64, (batch_stream_waves_per_eu<T, NK>())) void k_theta_stream_batch(
    T* pool, const BatchInst* __restrict__ insts,
                                                                   const ThItem* __restrict__ items, int nitems,
                                                                   const double* __restrict__ sig_pool,
                                                                   const double* __restrict__ kap_pool)
{
    typedef typename Vec16<T>::V VT;
    typedef StreamLayout<T, NK> L;
    constexpr int NW = NK / 16;
    constexpr int NT = NW * 64;
    constexpr int LD = L::LD;
    constexpr int VN = Vec16<T>::N;
    constexpr int NV = NK * NK / (NT * VN);

    extern __shared__ unsigned char smem_raw[];
    T* Xbase = reinterpret_cast<T*>(smem_raw);
    T* X = Xbase + L::PADR * LD;
    T* tk = Xbase + L::X_ELEMS;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
    for (int e = tid; e < L::PADR * LD; e += NT) {
        Xbase[e] = T(0);
        X[NK * LD + e] = T(0);
    }
    for (int e = tid; e < NK * L::PADC; e += NT) X[(e / L::PADC) * LD + NK + e % L::PADC] = T(0);

    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const ThItem item = items[it];
        const BatchInst I = insts[item.inst];
        T* base = pool + I.off;
        const double* sig = sig_pool + I.tab_off;
        const double* kap = kap_pool + I.tab_off;
        for (int g = 0; g < item.np; ++g) {
            const long pl = (long)item.plane0 + g;
            const VT* src = reinterpret_cast<const VT*>(base + pl * (long)NK * NK);
            VT xr[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) xr[v] = src[tid + v * NT];
            double kraw = 0.0;
            if (I.two_body && tid < 2 * NK) {
                const int i1 = (int)(pl / I.nx), i2 = (int)(pl % I.nx);
                const int ell = (i1 - i2 + I.nx) % I.nx;
                const int d = tid - NK, ad = d < 0 ? -d : d;
                kraw = kap[(long)ell * NK + min(max(ad, 1), NK - 1)];
            }
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const int e = (tid + v * NT) * VN;
                *reinterpret_cast<VT*>(X + (e / NK) * LD + e % NK) = xr[v];
            }
            if (tid < 2 * NK) {
                const int d = tid - NK, ad = d < 0 ? -d : d;
                tk[tid] = (I.two_body && ad > 0 && ad < NK) ? sgnval(d, T(kraw)) : T(0);
            }
            __syncthreads();
            if (I.two_body)
                stream_plane<T, NK, true, 3, 1>(nullptr, base, I.nx, pl, sig, sig, I.band, I.tau, X, tk, lane, w, 0);
            else
                stream_plane<T, NK, false, 3, 1>(nullptr, base, I.nx, pl, sig, sig, I.band, I.tau, X, tk, lane, w,
                                                 0);
        }
    }
}

template <typename T, int NK>
hipError_t go_stream_batch(T* pool, const BatchInst* insts, const ThItem* items, int nitems, const double* sig,
                           const double* kap, int grid, hipStream_t st)
{
    auto kf = k_theta_stream_batch<T, NK>;
    const size_t sm = StreamLayout<T, NK>::bytes;
    hipError_t e = hipFuncSetAttribute((const void*)kf, hipFuncAttributeMaxDynamicSharedMemorySize, (int)sm);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(kf, dim3(grid), dim3(NK / 16 * 64), sm, st, pool, insts, items, nitems, sig, kap);
    return hipGetLastError();
}

}  // namespace

bool theta_stream_ok(const ThetaArgs& a)
{
    if (a.precision == WIG2_BF16X2) return theta_stream_bf16_ok(a);
    const bool nk_ok = a.nk == 32 || a.nk == 48 || a.nk == 64 || a.nk == 96 || a.nk == 128;
    return nk_ok && !a.ksem && a.band >= 0 && a.band <= kStreamBand &&
           (a.precision == WIG2_FP64 || a.precision == WIG2_FP32);
}

template <typename T>
hipError_t launch_theta_stream(const ThetaArgs& a, const T* x, const T* y, T* out, int form,
                               double tau, hipStream_t st)
{
    if (!theta_stream_ok(a) || (form == 2 && !y)) return hipErrorNotSupported;
    if (a.precision == WIG2_BF16X2) {
        if constexpr (sizeof(T) == 4)
            return launch_theta_stream_bf16(a, x, y, out, form, tau, st);
        else
            return hipErrorNotSupported;
    }
    switch (a.nk) {
    case 32: return go_stream_nk<T, 32>(a, x, y, out, form, tau, st);
    case 48: return go_stream_nk<T, 48>(a, x, y, out, form, tau, st);
    case 64: return go_stream_nk<T, 64>(a, x, y, out, form, tau, st);
    case 96: return go_stream_nk<T, 96>(a, x, y, out, form, tau, st);
    case 128: return go_stream_nk<T, 128>(a, x, y, out, form, tau, st);
    default: return hipErrorNotSupported;
    }
}

bool batch_stream_nk_ok(int nk, int elem_bytes)
{
    (void)elem_bytes;
    return nk == 32 || nk == 48 || nk == 64 || nk == 96 || nk == 128;
}

// The streaming kernel is the faster one at every plane size it supports
// (measured on MI355X, Strang steps of nx^2 nk^2 with a one-mode V_ext and
// the pair term, FP64 and FP32, nk = 32 .. 128: 1.1-1.7x the general kernel).
bool theta_stream_preferred(int nk, int elem_bytes)
{
    return batch_stream_nk_ok(nk, elem_bytes);
}

template <typename T>
hipError_t launch_theta_stream_batch(T* pool, const BatchInst* insts, const ThItem* items, int nitems,
                                     const double* sig_pool, const double* kap_pool, int nk, int grid,
                                     hipStream_t st)
{
    if (nitems == 0) return hipSuccess;
    if (!batch_stream_nk_ok(nk, sizeof(T))) return hipErrorInvalidValue;
    switch (nk) {
    case 32: return go_stream_batch<T, 32>(pool, insts, items, nitems, sig_pool, kap_pool, grid, st);
    case 48: return go_stream_batch<T, 48>(pool, insts, items, nitems, sig_pool, kap_pool, grid, st);
    case 64: return go_stream_batch<T, 64>(pool, insts, items, nitems, sig_pool, kap_pool, grid, st);
    case 96: return go_stream_batch<T, 96>(pool, insts, items, nitems, sig_pool, kap_pool, grid, st);
    case 128: return go_stream_batch<T, 128>(pool, insts, items, nitems, sig_pool, kap_pool, grid, st);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_theta_stream_batch<double>(double*, const BatchInst*, const ThItem*, int, const double*,
                                                      const double*, int, int, hipStream_t);
template hipError_t launch_theta_stream_batch<float>(float*, const BatchInst*, const ThItem*, int, const double*,
                                                     const double*, int, int, hipStream_t);

template hipError_t launch_theta_stream<double>(const ThetaArgs&, const double*, const double*,
                                                double*, int, double, hipStream_t);
template hipError_t launch_theta_stream<float>(const ThetaArgs&, const float*, const float*, float*,
                                               int, double, hipStream_t);

}  // namespace wig2
