// Box two-body operator Theta_12 (Sec. 3.2.2): the Poisson-summation route
// through a y-lattice, the potential difference D_V and the two-body tensor,
// evaluated as four real matrix products per momentum plane on the matrix
// cores.  For the plane F = f(x_i1, x_i2, ., .) (nk x nk) and the complex
// tables G[y][n] = int_{P} e^{2 i p y/hbar} ell_n(p) dp (ell_n the cell-wise
// Lagrange cardinal of node n) and B[n][y] = e^{-2 i p_n y/hbar},
//   Ft = G F G^T                      (transform of the cell interpolant)
//   H  = D_l o Ft,  D_l(y1, y2) = c (V12(r + y1 - y2) - V12(r - y1 + y2))
//   Theta_12 F = Im(B H B^T),         r = x_i1 - x_i2, c = dy^2/(pi^2 hbar^3)
// with the complex products written as real ones on stacked operands:
//   stage A  R  = X WA            X = u + beta v, R = [Re | Im] (nk x 2ny)
//   stage B  H' = WB R'           R' = R as (2nk x ny), rows Re/Im interleaved;
//                                 epilogue H = D_l o H', H = [H_re; H_im]
//   stage C  Q' = WC H            Q' (2nk x ny), rows Re/Im interleaved
//   stage D  out += alpha Q'' WD  Q'' = Q' as (nk x 2ny) = [Q_re | Q_im]
// Stages A and D act on the stacked planes of a chunk as one tall product
// (the shared table on the right); stages B and C apply a shared table on
// the left of every plane's block.  24 nk flops per point in all.
//
// Kernel: one 256-thread workgroup per (matrix, 64-row block) work item,
// walking the column blocks of that row block; 2 x 2 waves, each with a
// (TM/2) x (TN/2) piece of the tile on 16x16x4 matrix-core instructions;
// K in steps of 16 through double-buffered LDS, the next step's global
// loads in flight during the current step's products.  Work items of one
// plane go to one XCD (the per-plane operand is then fetched into one L2).
#include "common.h"
#include "mfma.h"

#include <algorithm>

namespace wig2 {
namespace {
using namespace mf;

constexpr int kKT = 16;  // K per LDS step

template <typename T, int TM, int TN>
struct GemmLds {
    static constexpr int LA = kKT + 1;        // A tile pitch (TM rows of kKT)
    static constexpr int LB = TN + 2;         // B tile pitch (kKT rows of TN)
    static constexpr int A_ELEMS = TM * LA;
    static constexpr int B_ELEMS = kKT * LB;
    static constexpr int STAGE = A_ELEMS + B_ELEMS;
    static constexpr size_t bytes = sizeof(T) * 2 * STAGE;
};

// Epilogues: 0 store, 1 multiply by the Toeplitz D_l and store, 2 C += alpha acc,
// 3 C = alpha acc.
template <typename T, int TM, int TN, int EPI, bool XPY>
__global__ __launch_bounds__(256) void k_sem12_gemm(const T* __restrict__ A, const T* __restrict__ A2,
                                                    double beta, long sA, const T* __restrict__ B, long sB,
                                                    T* __restrict__ C, long sC, int M, int N, int K,
                                                    long nbatch, const T* __restrict__ dtab, int nx, int ny,
                                                    long plane0, double alpha)
{
    typedef typename Acc<T>::V V;
    typedef GemmLds<T, TM, TN> L;
    constexpr int MT = TM / 32, NT = TN / 32;  // 16x16 blocks per wave
    constexpr int AV = TM * kKT / 256;         // A elements per thread per step
    constexpr int BV = kKT * TN / 256;
    __shared__ T lds[2 * L::STAGE];

    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    const int wm = wv >> 1, wn = wv & 1;
    const int li = lane & 15, lk = lane >> 4;
    const int rowtiles = M / TM;
    const long nwork = nbatch * rowtiles;
    // XCD-aware order: blocks k, k + 8, ... run on one XCD; give them
    // consecutive work items
    const long G = gridDim.x;
    const long xcd = blockIdx.x % 8, slot = blockIdx.x / 8;
    const long per = (G + 7) / 8;
    const long first = xcd * per + slot;

    for (long w = first; w < nwork; w += G) {
        const long b = w / rowtiles;
        const int r0 = (int)(w % rowtiles) * TM;
        const T* Ab = A + b * sA;
        const T* A2b = XPY ? A2 + b * sA : nullptr;
        const T* Bb = B + b * sB;
        T* Cb = C + b * sC;
        // D_l row of this plane's pair distance l = i1 - i2, and the row
        // offset of the tile within the y-lattice: r % ny = r0 % ny + (r - r0),
        // less ny once past it (tiles are at most 64 rows, ny >= 32)
        const T* drow = nullptr;
        int rmod0 = 0;
        if constexpr (EPI == 1) {
            const long pl = plane0 + b;
            const int l = (int)(pl / nx) - (int)(pl % nx);
            drow = dtab + (long)(l + nx - 1) * (2 * ny - 1) + ny - 1;
            rmod0 = r0 % ny;
        }
        for (int c0 = 0; c0 < N; c0 += TN) {
            V acc[MT][NT];
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j) acc[i][j] = V{0, 0, 0, 0};
            T ra[AV], rb[BV];
            // per-thread operand pointers, advanced by one K step per stage:
            // A element (r0 + tid / kKT + 256 v / kKT, tid % kKT + k0),
            // B element (tid / TN + 256 v / TN + k0, c0 + tid % TN)
            const T* pa = Ab + (long)(r0 + tid / kKT) * K + tid % kKT;
            const T* pa2 = XPY ? A2b + (long)(r0 + tid / kKT) * K + tid % kKT : nullptr;
            const T* pbb = Bb + (long)(tid / TN) * N + c0 + tid % TN;
            constexpr int AROWS = 256 / kKT, BROWS = 256 / TN;
            auto fetch = [&](int) {
#pragma unroll
                for (int v = 0; v < AV; ++v) {
                    ra[v] = pa[(long)v * AROWS * K];
                    if constexpr (XPY) ra[v] += T(beta) * pa2[(long)v * AROWS * K];
                }
#pragma unroll
                for (int v = 0; v < BV; ++v) rb[v] = pbb[(long)v * BROWS * N];
                pa += kKT;
                if constexpr (XPY) pa2 += kKT;
                pbb += (long)kKT * N;
            };
            auto stash = [&](int buf) {
                T* As = lds + buf * L::STAGE;
                T* Bs = As + L::A_ELEMS;
#pragma unroll
                for (int v = 0; v < AV; ++v) {
                    const int e = tid + 256 * v;
                    As[(e / kKT) * L::LA + e % kKT] = ra[v];
                }
#pragma unroll
                for (int v = 0; v < BV; ++v) {
                    const int e = tid + 256 * v;
                    Bs[(e / TN) * L::LB + e % TN] = rb[v];
                }
            };
            fetch(0);
            stash(0);
            __syncthreads();
            const int nks = K / kKT;
            for (int ks = 0; ks < nks; ++ks) {
                const int cur = ks & 1;
                if (ks + 1 < nks) fetch((ks + 1) * kKT);
                const T* As = lds + cur * L::STAGE;
                const T* Bs = As + L::A_ELEMS;
#pragma unroll
                for (int kk = 0; kk < kKT / 4; ++kk) {
                    T av[MT], bv[NT];
#pragma unroll
                    for (int i = 0; i < MT; ++i) av[i] = As[(wm * (TM / 2) + 16 * i + li) * L::LA + 4 * kk + lk];
#pragma unroll
                    for (int j = 0; j < NT; ++j) bv[j] = Bs[(4 * kk + lk) * L::LB + wn * (TN / 2) + 16 * j + li];
#pragma unroll
                    for (int i = 0; i < MT; ++i)
#pragma unroll
                        for (int j = 0; j < NT; ++j) acc[i][j] = mma(av[i], bv[j], acc[i][j]);
                }
                if (ks + 1 < nks) {
                    stash(cur ^ 1);
                }
                __syncthreads();
            }
            // epilogue
#pragma unroll
            for (int i = 0; i < MT; ++i)
#pragma unroll
                for (int j = 0; j < NT; ++j)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const int r = r0 + wm * (TM / 2) + 16 * i + acc_row<T>(lk, q);
                        const int c = c0 + wn * (TN / 2) + 16 * j + li;
                        const long gi = (long)r * N + c;
                        T v = acc[i][j][q];
                        if constexpr (EPI == 1) {
                            int rm = rmod0 + (r - r0);
                            rm = rm >= ny ? rm - ny : rm;
                            v *= drow[rm - c];
                            Cb[gi] = v;
                        } else if constexpr (EPI == 2) {
                            Cb[gi] += T(alpha) * v;
                        } else if constexpr (EPI == 3) {
                            Cb[gi] = T(alpha) * v;
                        } else {
                            Cb[gi] = v;
                        }
                    }
        }
    }
}

template <typename T, int TM, int TN, int EPI, bool XPY>
hipError_t go_gemm(const T* A, const T* A2, double beta, long sA, const T* B, long sB, T* C, long sC, int M,
                   int N, int K, long nbatch, const T* dtab, int nx, int ny, long plane0, double alpha,
                   int ncu, hipStream_t st)
{
    // a grid of at least 8 workgroups is a multiple of 8 (the XCD-aware
    // order in the kernel is a permutation of the block ids only then)
    const long nwork = nbatch * (M / TM);
    const long grid = nwork < 8 ? nwork : std::min<long>(nwork, 8L * ncu) / 8 * 8;
    hipLaunchKernelGGL((k_sem12_gemm<T, TM, TN, EPI, XPY>), dim3((unsigned)grid), dim3(256), 0, st, A, A2, beta,
                       sA, B, sB, C, sC, M, N, K, nbatch, dtab, nx, ny, plane0, alpha);
    return hipGetLastError();
}

// M, N multiples of 32 (TM, TN = 64 where they divide), K of 16.
template <typename T, int EPI, bool XPY>
hipError_t gemm(const T* A, const T* A2, double beta, long sA, const T* B, long sB, T* C, long sC, int M,
                int N, int K, long nbatch, const T* dtab, int nx, int ny, long plane0, double alpha, int ncu,
                hipStream_t st)
{
    if (M % 32 || N % 32 || K % kKT) return hipErrorInvalidValue;
    const bool m64 = M % 64 == 0, n64 = N % 64 == 0;
    if (m64 && n64)
        return go_gemm<T, 64, 64, EPI, XPY>(A, A2, beta, sA, B, sB, C, sC, M, N, K, nbatch, dtab, nx, ny,
                                            plane0, alpha, ncu, st);
    if (m64)
        return go_gemm<T, 64, 32, EPI, XPY>(A, A2, beta, sA, B, sB, C, sC, M, N, K, nbatch, dtab, nx, ny,
                                            plane0, alpha, ncu, st);
    if (n64)
        return go_gemm<T, 32, 64, EPI, XPY>(A, A2, beta, sA, B, sB, C, sC, M, N, K, nbatch, dtab, nx, ny,
                                            plane0, alpha, ncu, st);
    return go_gemm<T, 32, 32, EPI, XPY>(A, A2, beta, sA, B, sB, C, sC, M, N, K, nbatch, dtab, nx, ny, plane0,
                                        alpha, ncu, st);
}

}  // namespace

bool sem12_nk_ok(int nk) { return nk >= 32 && nk % 32 == 0 && nk <= 256; }

template <typename T>
hipError_t launch_sem12_pre(const Sem12Args& a, const T* u, const T* v, double beta, long plane0, long nplanes,
                            T* wr, T* wh, hipStream_t st)
{
    const int nk = a.nk, ny = a.nk;
    const long pp = (long)nk * nk;
    const T* WA = static_cast<const T*>(a.wa);
    const T* WB = static_cast<const T*>(a.wb);
    const T* WC = static_cast<const T*>(a.wc);
    const T* D = static_cast<const T*>(a.dtab);
    hipError_t e;
    // stage A: the chunk's planes stacked, (nplanes nk) x nk times WA (nk x 2ny)
    const T* u0 = u + plane0 * pp;
    const T* v0 = v ? v + plane0 * pp : nullptr;
    if (v)
        e = gemm<T, 0, true>(u0, v0, beta, 0, WA, 0, wr, 0, (int)(nplanes * nk), 2 * ny, nk, 1, nullptr, a.nx,
                             ny, plane0, 0.0, a.ncu, st);
    else
        e = gemm<T, 0, false>(u0, nullptr, 0.0, 0, WA, 0, wr, 0, (int)(nplanes * nk), 2 * ny, nk, 1, nullptr,
                              a.nx, ny, plane0, 0.0, a.ncu, st);
    if (e != hipSuccess) return e;
    // stage B: WB (2ny x 2nk) times R' (2nk x ny) per plane, then D_l
    e = gemm<T, 1, false>(WB, nullptr, 0.0, 0, wr, 2 * pp, wh, 2 * pp, 2 * ny, ny, 2 * nk, nplanes, D, a.nx, ny,
                          plane0, 0.0, a.ncu, st);
    if (e != hipSuccess) return e;
    // stage C: WC (2nk x 2ny) times H (2ny x ny) per plane, into wr
    return gemm<T, 0, false>(WC, nullptr, 0.0, 0, wh, 2 * pp, wr, 2 * pp, 2 * nk, ny, 2 * ny, nplanes, nullptr,
                             a.nx, ny, plane0, 0.0, a.ncu, st);
}

template <typename T>
hipError_t launch_sem12_post(const Sem12Args& a, const T* wr, T* out, double alpha, bool accumulate, long plane0,
                             long nplanes, hipStream_t st)
{
    const int nk = a.nk, ny = a.nk;
    const long pp = (long)nk * nk;
    const T* WD = static_cast<const T*>(a.wd);
    // stage D: Q'' (nplanes nk x 2ny) times WD (2ny x nk), scaled, onto or into out
    if (accumulate)
        return gemm<T, 2, false>(wr, nullptr, 0.0, 0, WD, 0, out + plane0 * pp, 0, (int)(nplanes * nk), nk, 2 * ny,
                                 1, nullptr, a.nx, ny, plane0, alpha, a.ncu, st);
    return gemm<T, 3, false>(wr, nullptr, 0.0, 0, WD, 0, out + plane0 * pp, 0, (int)(nplanes * nk), nk, 2 * ny, 1,
                             nullptr, a.nx, ny, plane0, alpha, a.ncu, st);
}

template <typename T>
__global__ __launch_bounds__(256) void k_sem12_add(const T* __restrict__ acc, T* __restrict__ out, long n)
{
    for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) out[i] += acc[i];
}

template <typename T>
hipError_t launch_sem12_add(const T* acc, T* out, long n, int ncu, hipStream_t st)
{
    const long grid = std::max<long>(1, std::min<long>((n + 255) / 256, 16L * ncu));
    hipLaunchKernelGGL(k_sem12_add<T>, dim3((unsigned)grid), dim3(256), 0, st, acc, out, n);
    return hipGetLastError();
}

template hipError_t launch_sem12_add<double>(const double*, double*, long, int, hipStream_t);
template hipError_t launch_sem12_add<float>(const float*, float*, long, int, hipStream_t);
template hipError_t launch_sem12_pre<double>(const Sem12Args&, const double*, const double*, double, long, long,
                                             double*, double*, hipStream_t);
template hipError_t launch_sem12_pre<float>(const Sem12Args&, const float*, const float*, double, long, long,
                                            float*, float*, hipStream_t);
template hipError_t launch_sem12_post<double>(const Sem12Args&, const double*, double*, double, bool, long, long,
                                              hipStream_t);
template hipError_t launch_sem12_post<float>(const Sem12Args&, const float*, float*, double, bool, long, long,
                                             hipStream_t);

}  // namespace wig2
