// FP64 reductions over the 4-D state: per-plane moments for the observables
// (Sec. 2.2 densities, Sec. 5 energy and norms, the reduced Wigner function
// of Sec. 5.2) and the mean-field potential update (Sec. 2.2-2.3).
//
// Every sum is a fixed-order tree (wavefront shuffles, then LDS), so results
// are bitwise reproducible run to run.  States may be FP32; accumulation is
// always FP64.
#include "common.h"

#include <cmath>

namespace wig2 {
namespace {

__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    return v;
}

// One workgroup (256 threads, 4 waves) per plane.  Wave w handles rows
// n1 = w, w+4, ...; lanes stride over n2.  With `rows` the row sums are
// reduced per row (the reduced Wigner function needs them); without, each
// lane keeps its weighted partial moments and the wave reduces once.
template <typename T>
__global__ __launch_bounds__(256) void k_plane_moments(const T* __restrict__ f, int nk,
                                                       const double* __restrict__ p,
                                                       const double* __restrict__ w,
                                                       double inv2m, double* __restrict__ s0,
                                                       double* __restrict__ skin,
                                                       double* __restrict__ s2,
                                                       double* __restrict__ rows)
{
    __shared__ double red[3][4];
    const long pl = blockIdx.x;
    const T* F = f + pl * (long)nk * nk;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    double a0 = 0.0, ak = 0.0, a2 = 0.0;
    if (!rows && 256 % (nk / 2) == 0) {
        // no per-row sums wanted, and nk / 2 divides the 256 threads: each
        // thread always reads the same pair of columns n2, n2 + 1 (one
        // vector) and accumulates over its rows the row-weighted sums
        //   r0 = sum w1 v,  rk = sum w1 p1^2 v,  r2 = sum w1 v^2,
        // the column weights entering once at the end
        typedef T T2 __attribute__((ext_vector_type(2)));
        const T2* F2 = reinterpret_cast<const T2*>(F);
        const int hk = nk / 2, half = nk * nk / 2;
        const int n2 = 2 * ((int)threadIdx.x % hk);
        const int rstep = 256 / hk;
        double r0[2] = {0.0, 0.0}, rk[2] = {0.0, 0.0}, r2[2] = {0.0, 0.0};
        int n1 = (int)threadIdx.x / hk;
#pragma unroll 4
        for (int e = threadIdx.x; e < half; e += 256, n1 += rstep) {
            const T2 v2 = F2[e];
            const double w1 = w[n1], wp1 = w1 * p[n1] * p[n1];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double v = (double)v2[h];
                const double t = w1 * v;
                r0[h] += t;
                rk[h] += wp1 * v;
                r2[h] += t * v;
            }
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const double w2 = w[n2 + h], pp2 = p[n2 + h] * p[n2 + h];
            a0 += w2 * r0[h];
            ak += w2 * (rk[h] + pp2 * r0[h]) * inv2m;
            a2 += w2 * r2[h];
        }
        a0 = wave_sum(a0);
        ak = wave_sum(ak);
        a2 = wave_sum(a2);
    } else if (!rows) {
        // no per-row sums wanted: every moment is a weighted sum of the
        // thread's own terms (pairs of neighbours in n2, read as one vector),
        // reduced once per wave at the end
        typedef T T2 __attribute__((ext_vector_type(2)));
        const T2* F2 = reinterpret_cast<const T2*>(F);
        const int half = nk * nk / 2;
#pragma unroll 4
        for (int e = threadIdx.x; e < half; e += 256) {
            const T2 v2 = F2[e];
            const int n1 = (2 * e) / nk, n2 = (2 * e) % nk;
            const double w1 = w[n1], pp1 = p[n1] * p[n1];
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const double v = (double)v2[h];
                const double ww = w1 * w[n2 + h] * v;
                a0 += ww;
                ak += ww * (pp1 + p[n2 + h] * p[n2 + h]) * inv2m;
                a2 += ww * v;
            }
        }
        a0 = wave_sum(a0);
        ak = wave_sum(ak);
        a2 = wave_sum(a2);
    }
    for (int n1 = wv; rows && n1 < nk; n1 += 4) {
        double r0 = 0.0, rp = 0.0, rq = 0.0;
        for (int n2 = lane; n2 < nk; n2 += 64) {
            const double v = (double)F[(long)n1 * nk + n2];
            const double wv2 = w[n2] * v;
            r0 += wv2;
            rp += wv2 * p[n2] * p[n2];
            rq += wv2 * v;
        }
        r0 = wave_sum(r0);
        rp = wave_sum(rp);
        rq = wave_sum(rq);
        if (lane == 0) {
            if (rows) rows[pl * nk + n1] = r0;
            a0 += w[n1] * r0;
            ak += w[n1] * (p[n1] * p[n1] * r0 + rp) * inv2m;
            a2 += w[n1] * rq;
        }
    }
    if (lane == 0) {
        red[0][wv] = a0;
        red[1][wv] = ak;
        red[2][wv] = a2;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        s0[pl] = (red[0][0] + red[0][1]) + (red[0][2] + red[0][3]);
        if (skin) skin[pl] = (red[1][0] + red[1][1]) + (red[1][2] + red[1][3]);
        if (s2) s2[pl] = (red[2][0] + red[2][1]) + (red[2][2] + red[2][3]);
    }
}

__global__ void k_reduce_rows(const double* __restrict__ rows, int nx, int nk, double dx,
                              double* __restrict__ f1)
{
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long)nx * nk) return;
    const int i1 = (int)(id / nk), n1 = (int)(id % nk);
    double s = 0.0;
    for (int i2 = 0; i2 < nx; ++i2) s += rows[((long)i1 * nx + i2) * nk + n1];
    f1[id] = dx * s;
}

// Hedin-Lundqvist potential in atomic units (a_B = 1): g_D = 0.985 n0^{1/3}
// makes the exchange part 0.985 n^{1/3} and the correlation part
// 0.985 * 0.034 ln(1 + 18.37 n^{1/3}); density clamped at zero.
__device__ inline double hl_potential(double n)
{
    const double c = cbrt(n > 0.0 ? n : 0.0);
    return 0.985 * c + 0.985 * 0.034 * log(1.0 + 18.37 * c);
}

// Densities and effective potentials for both particles (one block).
__global__ void k_meanfield_potential(MeanFieldArgs a, const double* __restrict__ s0,
                                      const double* __restrict__ s0b, double tau_b)
{
    const int nx = a.nx;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        double d1 = 0.0, d2 = 0.0;
        for (int j = 0; j < nx; ++j) {
            double v1 = s0[(long)i * nx + j], v2 = s0[(long)j * nx + i];
            if (s0b) {
                v1 += tau_b * s0b[(long)i * nx + j];
                v2 += tau_b * s0b[(long)j * nx + i];
            }
            d1 += v1;
            d2 += v2;
        }
        a.dens[i] = a.dx * d1;
        a.dens[nx + i] = a.dx * d2;
    }
    __syncthreads();
    const double xc0 = a.xc ? hl_potential(a.xc_n0) : 0.0;
    for (int i = threadIdx.x; i < nx; i += blockDim.x) {
        for (int pj = 0; pj < 2; ++pj) {
            const double* n = a.dens + pj * nx;
            double h = 0.0;
            for (int j = 0; j < nx; ++j) h += a.v12pair[(long)i * nx + j] * n[j];
            double v = a.lambda * a.dx * h;
            if (a.xc) v += hl_potential(a.n_scale * n[i]) - xc0;
            a.veff[pj * nx + i] = v;
        }
    }
}

// sig_j[i][m] = sig_ext[i][m] + (2/hbar)(1/nx) sum_k V_j(x_k) sin(2 pi m (i-k)/nx), 2m < nx.
__global__ void k_meanfield_symbols(MeanFieldArgs a, double* __restrict__ sig1,
                                    double* __restrict__ sig2)
{
    const int nx = a.nx, nk = a.nk;
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long)nx * nk) return;
    const int i = (int)(id / nk), m = (int)(id % nk);
    double h1 = 0.0, h2 = 0.0;
    if (m > 0 && 2 * m < nx) {
        const double* st = a.sintab + (long)m * nx;
        for (int k = 0; k < nx; ++k) {
            const double s = st[(i - k + nx) % nx];
            h1 += a.veff[k] * s;
            h2 += a.veff[nx + k] * s;
        }
        const double c = 2.0 / (a.hbar * nx);
        h1 *= c;
        h2 *= c;
    }
    sig1[id] = a.sig_ext[id] + h1;
    sig2[id] = a.sig_ext[id] + h2;
}

// Box mean field (Sec. 3.2.1): the SEM matrices of V_ext + V_eff,j.  The SEM
// single-body operator is linear in the potential, and its kernel factorises
// over the node distance d = i - l (tables from the host):
//   K_j[i][n][s N + k] = kext[i][n][s N + k]
//                        + pref sum_l V_j(x_l) Im(E[d][n][s] Q[d][k]).
template <typename T>
__global__ __launch_bounds__(256) void k_meanfield_sem(SemMfArgs a, T* __restrict__ k1t, T* __restrict__ k2t)
{
    const int nx = a.nx, nk = a.nk, N = a.nodes, M = nk / N;
    const long id = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (id >= (long)nx * nk * nk) return;
    const int i = (int)(id / ((long)nk * nk));
    const int rem = (int)(id % ((long)nk * nk));
    const int n = rem / nk, c = rem % nk, s = c / N, k = c % N;
    double acc1 = 0.0, acc2 = 0.0;
    for (int l = 0; l < nx; ++l) {
        const int d = i - l + nx - 1;
        const double* e = a.E + 2 * (((long)d * nk + n) * M + s);
        const double* q = a.Q + 2 * ((long)d * N + k);
        const double im = e[0] * q[1] + e[1] * q[0];
        acc1 += a.veff[l] * im;
        acc2 += a.veff[nx + l] * im;
    }
    const double v1 = a.kext[id] + a.pref * acc1, v2 = a.kext[id] + a.pref * acc2;
    a.k1[id] = v1;
    a.k2[id] = v2;
    if (k1t) {
        k1t[id] = T(v1);
        k2t[id] = T(v2);
    }
}

}  // namespace

hipError_t launch_meanfield_potential(const MeanFieldArgs& a, const double* s0, const double* s0b, double tau_b,
                                      hipStream_t st)
{
    hipLaunchKernelGGL(k_meanfield_potential, dim3(1), dim3(256), 0, st, a, s0, s0b, tau_b);
    return hipGetLastError();
}

hipError_t launch_meanfield_sem(const SemMfArgs& a, float* k1f, float* k2f, hipStream_t st)
{
    const long n = (long)a.nx * a.nk * a.nk;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_meanfield_sem<float>, dim3(nb), dim3(256), 0, st, a, k1f, k2f);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_plane_moments(const T* f, int nx, int nk, const double* p_dev,
                                const double* w_dev, double inv2m, double* s0, double* skin,
                                double* s2, double* rows, hipStream_t st)
{
    const unsigned np = (unsigned)((long)nx * nx);
    hipLaunchKernelGGL((k_plane_moments<T>), dim3(np), dim3(256), 0, st, f, nk, p_dev, w_dev, inv2m,
                       s0, skin, s2, rows);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(const double* rows, int nx, int nk, double dx, double* f1,
                              hipStream_t st)
{
    const long n = (long)nx * nk;
    hipLaunchKernelGGL(k_reduce_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, rows,
                       nx, nk, dx, f1);
    return hipGetLastError();
}

hipError_t launch_meanfield(const MeanFieldArgs& a, const double* s0, const double* s0b,
                            double tau_b, double* sig1, double* sig2, hipStream_t st)
{
    hipLaunchKernelGGL(k_meanfield_potential, dim3(1), dim3(256), 0, st, a, s0, s0b, tau_b);
    const long n = (long)a.nx * a.nk;
    hipLaunchKernelGGL(k_meanfield_symbols, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st,
                       a, sig1, sig2);
    return hipGetLastError();
}

template hipError_t launch_plane_moments<double>(const double*, int, int, const double*,
                                                 const double*, double, double*, double*, double*,
                                                 double*, hipStream_t);
template hipError_t launch_plane_moments<float>(const float*, int, int, const double*,
                                                const double*, double, double*, double*, double*,
                                                double*, hipStream_t);

}  // namespace wig2
