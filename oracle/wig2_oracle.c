/*
 * wig2_oracle.c -- plain FP64 CPU reference for one time step of the two-body
 * Wigner equation (Liang & Xiong, arXiv:2511.11354).
 *
 * TEST INFRASTRUCTURE ONLY: used by tests/, the smoke check and the benchmark's
 * CPU-baseline leg; never by the product library.  Shares no code with the HIP
 * path.  Straight loops in FP64, OpenMP only over independent outer indices.
 *
 * Sign convention (reading of the paper, see design notes): the pseudo-
 * differential operator carries the prefactor i/hbar of the mean-field Wigner
 * equation (Sec. 2.3, eq. sWigner, and the Wigner kernel, eq. decomposition).
 * The single-body pseudo-difference formula (Sec. 3.1.1, eq. Hartree_FSM) is
 * printed with 1/(i hbar); with that factor it is the negative of the paper's
 * own closed form in Sec. 5.1.1, so the first-principles sign is used here.
 * The two-body pseudo-difference formula (Sec. 3.1.2, eq. two_body_FSM) is
 * consistent as printed.
 *
 * Parity unpinned: or_hl (the Hedin-Lundqvist functional) only.  Every other
 * routine is pinned by tests/test_oracle_pins.py to closed forms, exact
 * identities, convergence rates or brute force.
 */
#include "wig2_oracle.h"

#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_PI 3.14159265358979323846264338327950288

int or_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

static double or_len(const or_grid* g) { return g->x_max - g->x_min; }

/* Spatial spacing.  Torus: nx distinct points, dx = L/nx (Sec. 3.1).
 * Box: nx nodes including both ends, dx = L/(nx-1) (Sec. 4.1). */
double or_dx(const or_grid* g)
{
    return g->periodic ? or_len(g) / g->nx : or_len(g) / (g->nx - 1);
}

void or_xnodes(const or_grid* g, double* x)
{
    double dx = or_dx(g);
    for (int i = 0; i < g->nx; ++i) x[i] = g->x_min + i * dx;
}

/* Momentum nodes and quadrature weights.
 * Torus (Sec. 3.1): dp = hbar*pi/L, p_n = (n - floor(nk/2)) dp, weight dp.
 * Box (Sec. 3.2, eq. spectral_representation / eq:base): the p-box
 * [-hbar k_max, hbar k_max] is cut into `cells` equal cells; each holds
 * N = nk/cells Chebyshev-Gauss nodes (roots of T_N), in increasing order.  The
 * weights integrate the cell's degree-(N-1) Chebyshev interpolant exactly,
 * which is Fejer's first rule scaled to the cell. */
void or_pnodes(const or_grid* g, double* p, double* w)
{
    int nk = g->nk;
    if (g->periodic) {
        double dp = g->hbar * OR_PI / or_len(g);
        for (int n = 0; n < nk; ++n) {
            p[n] = (n - nk / 2) * dp;
            w[n] = dp;
        }
        return;
    }
    int M = g->cells, N = nk / M;
    double pmax = g->hbar * g->k_max;
    double width = 2.0 * pmax / M;
    for (int s = 0; s < M; ++s) {
        double centre = -pmax + (s + 0.5) * width;
        for (int j = 0; j < N; ++j) {
            double th = (2.0 * j + 1.0) * OR_PI / (2.0 * N);
            double eta = -cos(th);
            double sum = 0.0;
            for (int k = 1; k <= N / 2; ++k)
                sum += cos(2.0 * k * th) / (4.0 * k * k - 1.0);
            p[s * N + j] = centre + 0.5 * width * eta;
            w[s * N + j] = 0.5 * width * (2.0 / N) * (1.0 - 2.0 * sum);
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Fourier symbols of the pseudo-difference operators (Sec. 3.1)             */
/* ------------------------------------------------------------------------ */

/* Single-body symbol of V_ext (Sec. 3.1.1).  V = sum_m Vhat_m e^{-2 pi i m x/L};
 * Vhat_m by the 2nk-point periodic trapezoid on y_j = x_min + j L/(2nk).
 * With the i/hbar prefactor the pair of modes +-m gives
 *   Theta_1 f(n) = (2/hbar) sum_{m>=1} sig_m(x) [f(n-m) - f(n+m)],
 *   sig_m(x) = -Im(Vhat_m e^{-2 pi i m x/L})
 *            = (1/2nk) sum_j V(y_j) sin(2 pi m (x - y_j)/L).
 * sig[i*nk + m], m = 0..nk-1, sig_0 = 0. */
void or_sigma_ext(const or_grid* g, const double* v_y, double* sig)
{
    int nx = g->nx, nk = g->nk, ny = 2 * nk;
    double L = or_len(g), dx = or_dx(g);
#pragma omp parallel for
    for (int i = 0; i < nx; ++i) {
        double x = g->x_min + i * dx;
        sig[(long)i * nk] = 0.0;
        for (int m = 1; m < nk; ++m) {
            double s = 0.0;
            for (int j = 0; j < ny; ++j) {
                double y = g->x_min + j * L / ny;
                s += v_y[j] * sin(2.0 * OR_PI * m * (x - y) / L);
            }
            sig[(long)i * nk + m] = s / ny;
        }
    }
}

/* Fourier modes of an even pair potential V12(r) on the torus (Sec. 3.1.2):
 * Vhat_m = (1/2nk) sum_j V12(r_j) cos(2 pi m r_j / L), r_j = -L/2 + j L/(2nk),
 * m = 0..nk-1 (the 2nk-point rule of the paper with the endpoint counted once).*/
void or_vhat12(const or_grid* g, const double* v12_r, double* vhat)
{
    int nk = g->nk, ny = 2 * nk;
    double L = or_len(g);
    for (int m = 0; m < nk; ++m) {
        double s = 0.0;
        for (int j = 0; j < ny; ++j) {
            double r = -0.5 * L + j * L / ny;
            s += v12_r[j] * cos(2.0 * OR_PI * m * r / L);
        }
        vhat[m] = s / ny;
    }
}

/* Symbol of a density-driven potential sampled on the x-grid (Sec. 3.1.1 with
 * the x-grid DFT): only |m| < nx/2 are resolved, the Nyquist mode is dropped.
 *   sig_m(x_i) = (1/nx) sum_j V(x_j) sin(2 pi m (x_i - x_j)/L). */
void or_sigma_hxc(const or_grid* g, const double* v_x, double* sig)
{
    int nx = g->nx, nk = g->nk;
    double L = or_len(g), dx = or_dx(g);
#pragma omp parallel for
    for (int i = 0; i < nx; ++i) {
        double xi = g->x_min + i * dx;
        sig[(long)i * nk] = 0.0;
        for (int m = 1; m < nk; ++m) {
            double s = 0.0;
            if (2 * m < nx) {
                for (int j = 0; j < nx; ++j) {
                    double xj = g->x_min + j * dx;
                    s += v_x[j] * sin(2.0 * OR_PI * m * (xi - xj) / L);
                }
                s /= nx;
            }
            sig[(long)i * nk + m] = s;
        }
    }
}

/* Single-particle densities (Sec. 2.2): n_1(x1) = int f dx2 dp1 dp2 and
 * n_2(x2) = int f dx1 dp1 dp2, as plain weighted sums. */
void or_densities(const or_grid* g, const double* f, double* n1, double* n2)
{
    int nx = g->nx, nk = g->nk;
    double dx = or_dx(g);
    double* p = malloc(sizeof(double) * nk);
    double* w = malloc(sizeof(double) * nk);
    or_pnodes(g, p, w);
    for (int i = 0; i < nx; ++i) { n1[i] = 0.0; n2[i] = 0.0; }
    for (int i1 = 0; i1 < nx; ++i1)
        for (int i2 = 0; i2 < nx; ++i2) {
            const double* F = f + ((long)i1 * nx + i2) * nk * nk;
            double s = 0.0;
            for (int a = 0; a < nk; ++a)
                for (int b = 0; b < nk; ++b) s += w[a] * w[b] * F[a * nk + b];
            n1[i1] += dx * s;
            n2[i2] += dx * s;
        }
    free(p);
    free(w);
}

/* Hedin-Lundqvist exchange-correlation potential (Sec. 2.2) in atomic units
 * (hbar = e = m = 4 pi eps0 = 1, a_B = 1).  Then g_D = 0.985 n0^{1/3} and
 *   V_xc(n) = 0.985 n^{1/3} + 0.985*0.034 ln(1 + 18.37 n^{1/3}),
 * signs as printed; the density is clamped at zero.
 * Parity unpinned: the paper prints no value of this functional to check it
 * against (its constants are 3-D physical-unit formulas). */
static double or_hl(double n)
{
    double c = cbrt(n > 0.0 ? n : 0.0);
    return 0.985 * c + 0.985 * 0.034 * log(1.0 + 18.37 * c);
}

/* Mean-field potential on the x-grid from a density (Sec. 2.3 and the two-body
 * truncation, Sec. 2.4):  V(x_i) = lambda * dx sum_j V12(x_i - x_j) n(x_j)
 *   + [xc] (V_xc(n_scale n(x_i)) - V_xc(n0)). */
void or_veff_hxc(const or_grid* g, const or_params* prm, const double* v12_pair,
                 const double* n, double* v)
{
    int nx = g->nx;
    double dx = or_dx(g);
    double* vh = NULL;
    if (prm->hartree == 1) {
        vh = malloc(sizeof(double) * nx);
        or_hartree_poisson(g, n, vh);
    }
    for (int i = 0; i < nx; ++i) {
        if (vh) {
            v[i] = prm->lambda * vh[i];
        } else {
            double s = 0.0;
            for (int j = 0; j < nx; ++j) s += v12_pair[(long)i * nx + j] * n[j];
            v[i] = prm->lambda * dx * s;
        }
        if (prm->xc) v[i] += or_hl(prm->n_scale * n[i]) - or_hl(prm->xc_n0);
    }
    free(vh);
}

/* Hartree potential of the neutralised 1-D Coulomb system on the torus
 * (Sec. 3.1.1, example of the neutralised ion background): with the Fourier
 * coefficients a_m = (1/nx) sum_j n(x_j) e^{2 pi i m x_j / L} of the density,
 * whose zero mode the background cancels,
 *   V_H(x_i) = sum_{0 < |m| < nx/2} (L^2 / (4 pi^2 m^2)) a_m e^{-2 pi i m x_i / L},
 * the solution of -V_H'' = n - mean(n) (the Nyquist mode is dropped, as for
 * the other density-driven symbols). */
void or_hartree_poisson(const or_grid* g, const double* n, double* v)
{
    int nx = g->nx;
    double L = or_len(g), dx = or_dx(g);
    for (int i = 0; i < nx; ++i) {
        double complex acc = 0.0;
        double xi = g->x_min + i * dx;
        for (int m = -(nx - 1) / 2; m <= (nx - 1) / 2; ++m) {
            if (m == 0 || 2 * abs(m) >= nx) continue;
            double complex am = 0.0;
            for (int j = 0; j < nx; ++j) am += n[j] * cexp(2.0 * I * OR_PI * m * (g->x_min + j * dx) / L);
            am /= nx;
            acc += L * L / (4.0 * OR_PI * OR_PI * m * m) * am * cexp(-2.0 * I * OR_PI * m * xi / L);
        }
        v[i] = creal(acc);
    }
}

/* Hartree potential of a box density by the zero-padded transform of
 * Sec. 3.2.1 (remark, eq. Hartree_approximation): the density, zero outside
 * the box, and V12 sampled at nu dx for nu in [-Nt/2, Nt/2) are transformed on
 * the padded grid of Nt = 3 nx points, multiplied and transformed back,
 *   V_H(x_m) = dx (1/Nt) sum_l Vt_l nt_l e^{2 pi i l m / Nt},
 *   Vt_l = sum_nu V12(nu dx) e^{-2 pi i l nu / Nt},  nt_l = sum_j n_j e^{-2 pi i l j / Nt}.
 * v12_pad[nu + Nt/2] = V12(nu dx). */
void or_hartree_padded(const or_grid* g, const double* v12_pad, const double* n, double* v)
{
    int nx = g->nx, nt = 3 * nx;
    double dx = or_dx(g);
    double complex* vt = malloc(sizeof(double complex) * nt);
    double complex* ntl = malloc(sizeof(double complex) * nt);
    for (int l = 0; l < nt; ++l) {
        double complex a = 0.0, b = 0.0;
        for (int nu = -nt / 2; nu < nt - nt / 2; ++nu)
            a += v12_pad[nu + nt / 2] * cexp(-2.0 * I * OR_PI * l * nu / nt);
        for (int j = 0; j < nx; ++j) b += n[j] * cexp(-2.0 * I * OR_PI * l * j / nt);
        vt[l] = a;
        ntl[l] = b;
    }
    for (int m = 0; m < nx; ++m) {
        double complex acc = 0.0;
        for (int l = 0; l < nt; ++l) acc += vt[l] * ntl[l] * cexp(2.0 * I * OR_PI * l * m / nt);
        v[m] = dx * creal(acc) / nt;
    }
    free(vt);
    free(ntl);
}

/* ------------------------------------------------------------------------ */
/* Theta application                                                         */
/* ------------------------------------------------------------------------ */

static double or_at(const double* F, int nk, int a, int b)
{
    if (a < 0 || a >= nk || b < 0 || b >= nk) return 0.0; /* f = 0 off the p-box */
    return F[a * nk + b];
}

/* Periodic Theta = Theta_1 + Theta_2 + Theta_12 on planes [plane0, plane0+n)
 * where plane = i1*nx + i2.  Direct sums over every shift m = 1..nk-1 whose
 * shifted index may lie in the box; values off the box are zero (Sec. 3.1).
 *   Theta_1  = (2/hbar) sum_m sig1_m(x_i1) [f(n1-m,n2) - f(n1+m,n2)]
 *   Theta_2  = (2/hbar) sum_m sig2_m(x_i2) [f(n1,n2-m) - f(n1,n2+m)]
 *   Theta_12 = (2/hbar) sum_m Vhat_m sin(2 pi m (i1-i2)/nx)
 *                              [f(n1-m,n2+m) - f(n1+m,n2-m)]
 * The last line is eq. two_body_FSM with the +-m modes of the even, real V12
 * combined. */
void or_theta_periodic(const or_grid* g, const double* sig1, const double* sig2,
                       const double* vhat12, int two_body,
                       long plane0, long nplanes, const double* f, double* out)
{
    int nx = g->nx, nk = g->nk;
    double c = 2.0 / g->hbar;
#pragma omp parallel
    {
        double* kap = malloc(sizeof(double) * nk);
#pragma omp for schedule(dynamic)
        for (long q = 0; q < nplanes; ++q) {
            long pl = plane0 + q;
            int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
            const double* F = f + pl * nk * nk;
            double* O = out + pl * nk * nk;
            const double* s1 = sig1 + (long)i1 * nk;
            const double* s2 = sig2 + (long)i2 * nk;
            for (int m = 0; m < nk; ++m)
                kap[m] = two_body ? vhat12[m] * sin(2.0 * OR_PI * m * (i1 - i2) / nx) : 0.0;
            for (int n1 = 0; n1 < nk; ++n1)
                for (int n2 = 0; n2 < nk; ++n2) {
                    double acc = 0.0;
                    for (int m = 1; m < nk; ++m) {
                        acc += s1[m] * (or_at(F, nk, n1 - m, n2) - or_at(F, nk, n1 + m, n2));
                        acc += s2[m] * (or_at(F, nk, n1, n2 - m) - or_at(F, nk, n1, n2 + m));
                        acc += kap[m] * (or_at(F, nk, n1 - m, n2 + m) - or_at(F, nk, n1 + m, n2 - m));
                    }
                    O[n1 * nk + n2] = c * acc;
                }
        }
        free(kap);
    }
}

/* Non-periodic single-body Theta with dense per-x matrices (Sec. 3.2.1):
 * out(n1,n2) = sum_a K1[i1][n1][a] f(a,n2) + sum_b K2[i2][n2][b] f(n1,b). */
void or_theta_dense(const or_grid* g, const double* K1, const double* K2,
                    long plane0, long nplanes, const double* f, double* out)
{
    int nx = g->nx, nk = g->nk;
#pragma omp parallel for schedule(dynamic)
    for (long q = 0; q < nplanes; ++q) {
        long pl = plane0 + q;
        int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
        const double* F = f + pl * nk * nk;
        double* O = out + pl * nk * nk;
        const double* A = K1 + (long)i1 * nk * nk;
        const double* B = K2 + (long)i2 * nk * nk;
        for (int n1 = 0; n1 < nk; ++n1)
            for (int n2 = 0; n2 < nk; ++n2) {
                double acc = 0.0;
                for (int a = 0; a < nk; ++a) acc += A[n1 * nk + a] * F[a * nk + n2];
                for (int b = 0; b < nk; ++b) acc += B[n2 * nk + b] * F[n1 * nk + b];
                O[n1 * nk + n2] = acc;
            }
    }
}

/* Chebyshev polynomial T_l(x) by the three-term recurrence. */
static double or_cheb(int l, double x)
{
    double t0 = 1.0, t1 = x;
    if (l == 0) return t0;
    for (int k = 2; k <= l; ++k) {
        double t2 = 2.0 * x * t1 - t0;
        t0 = t1;
        t1 = t2;
    }
    return t1;
}

/* Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_q. */
static void or_gauss_legendre(int q, double* x, double* w)
{
    for (int i = 0; i < q; ++i) {
        double z = cos(OR_PI * (i + 0.75) / (q + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (z * p1 - p0) / (z * z - 1.0);
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* SEM single-body matrix K[i][n][n'] (Sec. 3.2.1, eqs. nonlinear_Wigner_potential,
 * Chebyshev_PDO, basic_osc_int), with the first-principles sign i/hbar:
 *  1. V_W(x, q) ~ (2 dx/(pi hbar^2)) sum_j V(x_j) sin(2 q (x - x_j)/hbar)
 *     (Fourier transform of V replaced by the x-grid sum, periodic images
 *     ignored).
 *  2. On cell s, f(p') = sum_l b_{s,l} T_l(eta'), p' = dhat_s + |P|/2 eta',
 *     b_{s,l} = (2 - delta_l0)/N sum_k f(p_{s,k}) T_l(eta_k).
 *  3. int_{P_s} sin(2(p-p')z/hbar) T_l dp'
 *       = |P|/2 Im[ e^{2i(p - dhat_s) z/hbar} O_l(-|P| z/hbar) ],  z = x - x_j,
 *     O_l(zeta) = int_{-1}^{1} e^{i zeta eta} T_l(eta) d eta by Gauss-Legendre.
 * Assembled so that Theta_1 f(x_i, p_n) = sum_{n'} K[i][n][n'] f(p_{n'}). */
void or_sem_kernel(const or_grid* g, const double* v_x, double* K)
{
    int nx = g->nx, nk = g->nk, M = g->cells, N = nk / M;
    double hb = g->hbar, dx = or_dx(g);
    double pmax = hb * g->k_max, width = 2.0 * pmax / M;
    double* p = malloc(sizeof(double) * nk);
    double* w = malloc(sizeof(double) * nk);
    or_pnodes(g, p, w);
    double* eta = malloc(sizeof(double) * N);
    for (int j = 0; j < N; ++j) eta[j] = -cos((2.0 * j + 1.0) * OR_PI / (2.0 * N));
    /* O_l(zeta) for zeta = -|P| (d dx)/hbar, d = i - j in [-(nx-1), nx-1]. */
    int nd = 2 * nx - 1;
    double* Ore = malloc(sizeof(double) * nd * N);
    double* Oim = malloc(sizeof(double) * nd * N);
    for (int d = -(nx - 1); d <= nx - 1; ++d) {
        double zeta = -width * (d * dx) / hb;
        int q = 64;
        int need = (int)(fabs(zeta) + N + 32);
        if (need > q) q = need;
        double* gx = malloc(sizeof(double) * q);
        double* gw = malloc(sizeof(double) * q);
        or_gauss_legendre(q, gx, gw);
        for (int l = 0; l < N; ++l) {
            double re = 0.0, im = 0.0;
            for (int t = 0; t < q; ++t) {
                double T = or_cheb(l, gx[t]);
                re += gw[t] * cos(zeta * gx[t]) * T;
                im += gw[t] * sin(zeta * gx[t]) * T;
            }
            Ore[(d + nx - 1) * N + l] = re;
            Oim[(d + nx - 1) * N + l] = im;
        }
        free(gx);
        free(gw);
    }
    double pref = 2.0 * dx / (OR_PI * hb * hb);
#pragma omp parallel
    {
        double* A = malloc(sizeof(double) * M * N); /* A[s][l] for fixed (i,n) */
#pragma omp for
        for (int i = 0; i < nx; ++i) {
            double xi = g->x_min + i * dx;
            for (int n = 0; n < nk; ++n) {
                for (int s = 0; s < M; ++s) {
                    double dhat = -pmax + (s + 0.5) * width;
                    for (int l = 0; l < N; ++l) {
                        double acc = 0.0;
                        for (int j = 0; j < nx; ++j) {
                            double z = xi - (g->x_min + j * dx);
                            double ph = 2.0 * (p[n] - dhat) * z / hb;
                            double ore = Ore[(i - j + nx - 1) * N + l];
                            double oim = Oim[(i - j + nx - 1) * N + l];
                            /* Im[(cos ph + i sin ph)(ore + i oim)] */
                            acc += v_x[j] * (sin(ph) * ore + cos(ph) * oim);
                        }
                        A[s * N + l] = acc;
                    }
                }
                for (int s = 0; s < M; ++s)
                    for (int k = 0; k < N; ++k) {
                        double acc = 0.0;
                        for (int l = 0; l < N; ++l) {
                            double bl = (l == 0 ? 1.0 : 2.0) / N * or_cheb(l, eta[k]);
                            acc += A[s * N + l] * bl;
                        }
                        K[((long)i * nk + n) * nk + s * N + k] = pref * 0.5 * width * acc;
                    }
            }
        }
        free(A);
    }
    free(Ore);
    free(Oim);
    free(eta);
    free(p);
    free(w);
}

/* Spacing of the two-body y-lattice of the box (Sec. 3.2.2): dy = pi hbar / |P|
 * with |P| = 2 hbar k_max the length of the p-box, so that the y-sums below
 * are periodic in p with the period |P|. */
double or_sem12_dy(const or_grid* g) { return OR_PI / (2.0 * g->k_max); }

/* Non-periodic two-body operator Theta_12 by the spectral-element route of
 * Sec. 3.2.2 (Poisson summation in y, D_V, the two-body tensor
 * O_{s1 s2 l1 l2}), in the paper's order, with the readings below:
 *  1. Chebyshev coefficients of f on every cell pair (eq. spectral_representation):
 *       a_{s1 s2 l1 l2} = sum_{k1,k2} c_{l1 k1} c_{l2 k2} f(p_{s1,k1}, p_{s2,k2}),
 *       c_{lk} = (2 - delta_l0)/N T_l(eta_k).
 *  2. The two-body tensor contracted with a,
 *       Ft(y1, y2) = sum a_{s1 s2 l1 l2} O_{s1 s2 l1 l2}(y1, y2),
 *       O = prod_{j=1,2} (|P_s|/2) e^{2 i dhat_{s_j} y_j / hbar} O_{l_j}(|P_s| y_j / hbar),
 *     i.e. the integral of f(p1', p2') e^{2 i (p1' y1 + p2' y2)/hbar} over the
 *     p-box for the cell-wise interpolant.  The tensor is a product of one
 *     factor per particle, so the sum is taken one particle at a time.
 *  3. The potential difference D_V at r = x_i1 - x_i2:
 *       D(y1, y2) = V12(r + y1 - y2) - V12(r - y1 + y2).
 *  4. Theta_12(p1, p2) = (dy^2 / (pi^2 hbar^3))
 *       sum_{y1, y2} Im[ e^{-2 i (p1 y1 + p2 y2)/hbar} D(y1, y2) Ft(y1, y2) ].
 * Readings (the printed constants of this passage are garbled): with the
 * kernel e^{2 i p y / hbar} of the two-body tensor, the inverse transform of
 * the two-body Wigner kernel shifts V12 by the full y (not y/2), and the
 * prefactor follows from the pseudo-difference form of eq. two_body_FSM
 * (Theta_12 f = (2/(pi hbar^2)) int Vhat(2p'/hbar) sin(2 p' r / hbar)
 * f(p1 - p', p2 + p') dp', Vhat the Fourier transform of V12), whose sign
 * matches the closed form of Sec. 5.1.2.  Lattice: the nk midpoints
 * y_j = (j + 1/2 - nk/2) dy, j = 0..nk-1, symmetric under y -> -y (the sum is
 * then real term by term in pairs).
 * v12_tab[(l + nx - 1)(2 nk - 1) + (d + nk - 1)] = V12(l dx + d dy) for
 * l in [-(nx-1), nx-1], d in [-(nk-1), nk-1].  out = Theta_12 f on the planes
 * [plane0, plane0 + nplanes). */
void or_theta12_sem(const or_grid* g, const double* v12_tab, long plane0, long nplanes,
                    const double* f, double* out)
{
    int nx = g->nx, nk = g->nk, M = g->cells, N = nk / M, ny = nk;
    double hb = g->hbar, dy = or_sem12_dy(g);
    double pmax = hb * g->k_max, width = 2.0 * pmax / M;
    double* p = malloc(sizeof(double) * nk);
    double* w = malloc(sizeof(double) * nk);
    or_pnodes(g, p, w);
    double* y = malloc(sizeof(double) * ny);
    for (int j = 0; j < ny; ++j) y[j] = (j + 0.5 - 0.5 * ny) * dy;
    /* c[l][k] */
    double* cc = malloc(sizeof(double) * N * N);
    for (int l = 0; l < N; ++l)
        for (int k = 0; k < N; ++k) {
            double eta = -cos((2.0 * k + 1.0) * OR_PI / (2.0 * N));
            cc[l * N + k] = (l == 0 ? 1.0 : 2.0) / N * or_cheb(l, eta);
        }
    /* E[j][s N + l] = (|P|/2) e^{2 i dhat_s y_j / hbar} O_l(|P| y_j / hbar) */
    double complex* E = malloc(sizeof(double complex) * ny * nk);
    for (int j = 0; j < ny; ++j) {
        double zeta = width * y[j] / hb;
        int q = 64;
        int need = (int)(fabs(zeta) + N + 32);
        if (need > q) q = need;
        double* gx = malloc(sizeof(double) * q);
        double* gw = malloc(sizeof(double) * q);
        or_gauss_legendre(q, gx, gw);
        for (int l = 0; l < N; ++l) {
            double complex O = 0.0;
            for (int t = 0; t < q; ++t) O += gw[t] * cexp(I * zeta * gx[t]) * or_cheb(l, gx[t]);
            for (int sc = 0; sc < M; ++sc) {
                double dhat = -pmax + (sc + 0.5) * width;
                E[(long)j * nk + sc * N + l] = 0.5 * width * cexp(2.0 * I * dhat * y[j] / hb) * O;
            }
        }
        free(gx);
        free(gw);
    }
    double pref = dy * dy / (OR_PI * OR_PI * hb * hb * hb);
#pragma omp parallel
    {
        double* a = malloc(sizeof(double) * nk * nk);
        double* t = malloc(sizeof(double) * nk * nk);
        double complex* T2 = malloc(sizeof(double complex) * nk * ny);
        double complex* Ft = malloc(sizeof(double complex) * ny * ny);
        double complex* U = malloc(sizeof(double complex) * nk * ny);
#pragma omp for
        for (long pl = plane0; pl < plane0 + nplanes; ++pl) {
            int i1 = (int)(pl / nx), i2 = (int)(pl % nx);
            const double* F = f + pl * nk * nk;
            /* 1. coefficients: along p2 into t, then along p1 into a */
            for (int n1 = 0; n1 < nk; ++n1)
                for (int s2 = 0; s2 < M; ++s2)
                    for (int l2 = 0; l2 < N; ++l2) {
                        double acc = 0.0;
                        for (int k2 = 0; k2 < N; ++k2) acc += cc[l2 * N + k2] * F[n1 * nk + s2 * N + k2];
                        t[n1 * nk + s2 * N + l2] = acc;
                    }
            for (int s1 = 0; s1 < M; ++s1)
                for (int l1 = 0; l1 < N; ++l1)
                    for (int b = 0; b < nk; ++b) {
                        double acc = 0.0;
                        for (int k1 = 0; k1 < N; ++k1) acc += cc[l1 * N + k1] * t[(s1 * N + k1) * nk + b];
                        a[(s1 * N + l1) * nk + b] = acc;
                    }
            /* 2. tensor contraction, particle 2 then particle 1 */
            for (int al = 0; al < nk; ++al)
                for (int j2 = 0; j2 < ny; ++j2) {
                    double complex acc = 0.0;
                    for (int b = 0; b < nk; ++b) acc += a[al * nk + b] * E[(long)j2 * nk + b];
                    T2[al * ny + j2] = acc;
                }
            for (int j1 = 0; j1 < ny; ++j1)
                for (int j2 = 0; j2 < ny; ++j2) {
                    double complex acc = 0.0;
                    for (int al = 0; al < nk; ++al) acc += E[(long)j1 * nk + al] * T2[al * ny + j2];
                    Ft[j1 * ny + j2] = acc;
                }
            /* 3. times D_V */
            int l = i1 - i2;
            const double* vt = v12_tab + (long)(l + nx - 1) * (2 * nk - 1);
            for (int j1 = 0; j1 < ny; ++j1)
                for (int j2 = 0; j2 < ny; ++j2) {
                    int d = j1 - j2;
                    Ft[j1 * ny + j2] *= vt[d + nk - 1] - vt[-d + nk - 1];
                }
            /* 4. back to the momentum nodes, y1 then y2 */
            for (int n1 = 0; n1 < nk; ++n1)
                for (int j2 = 0; j2 < ny; ++j2) {
                    double complex acc = 0.0;
                    for (int j1 = 0; j1 < ny; ++j1)
                        acc += cexp(-2.0 * I * p[n1] * y[j1] / hb) * Ft[j1 * ny + j2];
                    U[n1 * ny + j2] = acc;
                }
            double* O = out + pl * nk * nk;
            for (int n1 = 0; n1 < nk; ++n1)
                for (int n2 = 0; n2 < nk; ++n2) {
                    double complex acc = 0.0;
                    for (int j2 = 0; j2 < ny; ++j2)
                        acc += U[n1 * ny + j2] * cexp(-2.0 * I * p[n2] * y[j2] / hb);
                    O[n1 * nk + n2] = pref * cimag(acc);
                }
        }
        free(a);
        free(t);
        free(T2);
        free(Ft);
        free(U);
    }
    free(p);
    free(w);
    free(y);
    free(cc);
    free(E);
}

/* ------------------------------------------------------------------------ */
/* Cubic B-spline advection (Sec. 4.1)                                       */
/* ------------------------------------------------------------------------ */

/* Dense LU with partial pivoting, row-major, in place. */
static int or_lu(int n, double* A, int* piv)
{
    for (int k = 0; k < n; ++k) {
        int pr = k;
        double best = fabs(A[(long)k * n + k]);
        for (int r = k + 1; r < n; ++r)
            if (fabs(A[(long)r * n + k]) > best) { best = fabs(A[(long)r * n + k]); pr = r; }
        if (best == 0.0) return -1;
        piv[k] = pr;
        if (pr != k)
            for (int c = 0; c < n; ++c) {
                double t = A[(long)k * n + c];
                A[(long)k * n + c] = A[(long)pr * n + c];
                A[(long)pr * n + c] = t;
            }
        for (int r = k + 1; r < n; ++r) {
            double l = A[(long)r * n + k] / A[(long)k * n + k];
            A[(long)r * n + k] = l;
            for (int c = k + 1; c < n; ++c) A[(long)r * n + c] -= l * A[(long)k * n + c];
        }
    }
    return 0;
}

static void or_lu_solve(int n, const double* LU, const int* piv, double* b)
{
    for (int k = 0; k < n; ++k) {
        int pr = piv[k];
        if (pr != k) { double t = b[k]; b[k] = b[pr]; b[pr] = t; }
    }
    for (int r = 0; r < n; ++r) {
        double s = b[r];
        for (int c = 0; c < r; ++c) s -= LU[(long)r * n + c] * b[c];
        b[r] = s;
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= LU[(long)r * n + c] * b[c];
        b[r] = s / LU[(long)r * n + r];
    }
}

/* Cubic B-spline weights on an interval, t in [0,1] (Sec. 4.1, B_nu):
 * coefficients of eta_{j-1}, eta_j, eta_{j+1}, eta_{j+2}. */
static void or_bweights(double t, double* w)
{
    w[0] = (1.0 - t) * (1.0 - t) * (1.0 - t) / 6.0;
    w[1] = (3.0 * t * t * t - 6.0 * t * t + 4.0) / 6.0;
    w[2] = (-3.0 * t * t * t + 3.0 * t * t + 3.0 * t + 1.0) / 6.0;
    w[3] = t * t * t / 6.0;
}

/* One advection sweep f <- f(x_d - s p_d / m) along dimension dim (1 or 2) on
 * the lines [line0, line0 + nlines).  A line is indexed by the other x index
 * and (n1, n2): line = (o*nk + n1)*nk + n2.
 * Torus: the periodic system (eta_{i-1} + 4 eta_i + eta_{i+1})/6 = g_i, solved
 * by dense LU; feet wrap into [x_min, x_min + L).
 * Box: the natural-boundary system A_nat with zero ghost values, unknowns
 * eta_{-1..nx}; feet outside [x_min, x_max] give zero. */
int or_advect(const or_grid* g, int dim, double s, long line0, long nlines,
              const double* f, double* out)
{
    int nx = g->nx, nk = g->nk;
    int per = g->periodic;
    int ns = per ? nx : nx + 2;
    double dx = or_dx(g), L = or_len(g);
    double* A = calloc((size_t)ns * ns, sizeof(double));
    int* piv = malloc(sizeof(int) * ns);
    double* p = malloc(sizeof(double) * nk);
    double* w = malloc(sizeof(double) * nk);
    or_pnodes(g, p, w);
    if (per) {
        for (int i = 0; i < nx; ++i) {
            A[(long)i * ns + i] += 4.0 / 6.0;
            A[(long)i * ns + (i + nx - 1) % nx] += 1.0 / 6.0;
            A[(long)i * ns + (i + 1) % nx] += 1.0 / 6.0;
        }
    } else {
        double h2 = 1.0 / (dx * dx);
        A[0] = h2; A[1] = -2.0 * h2; A[2] = h2;
        for (int r = 1; r <= nx; ++r) {
            A[(long)r * ns + r - 1] = 1.0 / 6.0;
            A[(long)r * ns + r] = 4.0 / 6.0;
            A[(long)r * ns + r + 1] = 1.0 / 6.0;
        }
        long r = nx + 1;
        A[r * ns + nx - 1] = h2; A[r * ns + nx] = -2.0 * h2; A[r * ns + nx + 1] = h2;
    }
    if (or_lu(ns, A, piv) != 0) { free(A); free(piv); free(p); free(w); return -1; }
    long stride = (dim == 1) ? (long)nx * nk * nk : (long)nk * nk;
#pragma omp parallel
    {
        double* b = malloc(sizeof(double) * ns);
#pragma omp for schedule(static)
        for (long q = 0; q < nlines; ++q) {
            long line = line0 + q;
            long o = line / ((long)nk * nk);
            int n1 = (int)((line / nk) % nk), n2 = (int)(line % nk);
            long base = (dim == 1) ? (o * nk * nk + (long)n1 * nk + n2)
                                   : (o * nx * nk * nk + (long)n1 * nk + n2);
            double v = p[dim == 1 ? n1 : n2] / g->mass;
            if (per) {
                for (int i = 0; i < nx; ++i) b[i] = f[base + i * stride];
            } else {
                b[0] = 0.0;
                for (int i = 0; i < nx; ++i) b[i + 1] = f[base + i * stride];
                b[nx + 1] = 0.0;
            }
            or_lu_solve(ns, A, piv, b);
            for (int i = 0; i < nx; ++i) {
                double foot = g->x_min + i * dx - s * v;
                double val = 0.0, wt[4];
                if (per) {
                    double u = (foot - g->x_min) / dx;
                    u -= nx * floor(u / nx);
                    int j = (int)floor(u);
                    double t = u - j;
                    if (j >= nx) j -= nx;
                    or_bweights(t, wt);
                    for (int k = 0; k < 4; ++k) val += wt[k] * b[((j + k - 1) % nx + nx) % nx];
                } else if (foot >= g->x_min && foot <= g->x_max) {
                    double u = (foot - g->x_min) / dx;
                    int j = (int)floor(u);
                    if (j > nx - 2) j = nx - 2;
                    double t = u - j;
                    or_bweights(t, wt);
                    for (int k = 0; k < 4; ++k) val += wt[k] * b[j + k]; /* eta_{j+k-1} */
                }
                out[base + i * stride] = val;
            }
        }
        free(b);
    }
    (void)L;
    free(A); free(piv); free(p); free(w);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Time step (Sec. 4.1, Lawson predictor-corrector; and the Strang split)    */
/* ------------------------------------------------------------------------ */

typedef struct {
    const or_grid* g;
    const or_params* prm;
    const or_tables* tb;
    double *sig1, *sig2;  /* periodic symbols actually used */
    double *n1, *n2, *v;
    double *K1, *K2;      /* box with a mean field: SEM matrices of V_ext + V_eff,j */
} or_ctx;

/* Rebuild the single-body symbols from the current density if the mean field
 * is on (torus only). */
static void or_symbols(or_ctx* c, const double* f)
{
    const or_grid* g = c->g;
    long nxk = (long)g->nx * g->nk;
    if (!g->periodic) {
        /* box: the SEM matrices of V_ext + V_eff,j (or_sem_kernel is linear in
         * the potential), the Hartree term the direct convolution with V12 */
        if (c->prm->lambda == 0.0 && !c->prm->xc) return;
        long nk2 = nxk * g->nk;
        double* kv = malloc(sizeof(double) * nk2);
        or_densities(g, f, c->n1, c->n2);
        or_veff_hxc(g, c->prm, c->tb->v12_pair, c->n1, c->v);
        or_sem_kernel(g, c->v, kv);
        for (long k = 0; k < nk2; ++k) c->K1[k] = c->tb->K[k] + kv[k];
        or_veff_hxc(g, c->prm, c->tb->v12_pair, c->n2, c->v);
        or_sem_kernel(g, c->v, kv);
        for (long k = 0; k < nk2; ++k) c->K2[k] = c->tb->K[k] + kv[k];
        free(kv);
        return;
    }
    memcpy(c->sig1, c->tb->sig_ext, sizeof(double) * nxk);
    memcpy(c->sig2, c->tb->sig_ext, sizeof(double) * nxk);
    if (c->prm->lambda == 0.0 && !c->prm->xc) return;
    double* sh = malloc(sizeof(double) * nxk);
    or_densities(g, f, c->n1, c->n2);
    or_veff_hxc(g, c->prm, c->tb->v12_pair, c->n1, c->v);
    or_sigma_hxc(g, c->v, sh);
    for (long k = 0; k < nxk; ++k) c->sig1[k] += sh[k];
    or_veff_hxc(g, c->prm, c->tb->v12_pair, c->n2, c->v);
    or_sigma_hxc(g, c->v, sh);
    for (long k = 0; k < nxk; ++k) c->sig2[k] += sh[k];
    free(sh);
}

static void or_theta_all(or_ctx* c, const double* f, double* out)
{
    const or_grid* g = c->g;
    long np = (long)g->nx * g->nx;
    if (g->periodic)
        or_theta_periodic(g, c->sig1, c->sig2, c->tb->vhat12, c->prm->two_body, 0, np, f, out);
    else {
        const int mf = c->prm->lambda != 0.0 || c->prm->xc;
        or_theta_dense(g, mf ? c->K1 : c->tb->K, mf ? c->K2 : c->tb->K, 0, np, f, out);
        if (c->prm->two_body && c->tb->v12_sem) {
            long n = np * g->nk * g->nk;
            double* t = malloc(sizeof(double) * n);
            or_theta12_sem(g, c->tb->v12_sem, 0, np, f, t);
            for (long k = 0; k < n; ++k) out[k] += t[k];
            free(t);
        }
    }
}

/* A_s = A^{x2}_s A^{x1}_s : x1 sweep first, then x2. */
static int or_advect_both(const or_grid* g, double s, double* f, double* tmp)
{
    long nl = (long)g->nx * g->nk * g->nk;
    if (or_advect(g, 1, s, 0, nl, f, tmp)) return -1;
    if (or_advect(g, 2, s, 0, nl, tmp, f)) return -1;
    return 0;
}

int or_step(const or_grid* g, const or_params* prm, const or_tables* tb,
            double* f, long nsteps)
{
    long N = (long)g->nx * g->nx * g->nk * g->nk;
    long nxk = (long)g->nx * g->nk;
    const int box_mf = !g->periodic && (prm->lambda != 0.0 || prm->xc);
    or_ctx c = {g, prm, tb, malloc(sizeof(double) * nxk), malloc(sizeof(double) * nxk),
                malloc(sizeof(double) * g->nx), malloc(sizeof(double) * g->nx),
                malloc(sizeof(double) * g->nx),
                box_mf ? malloc(sizeof(double) * nxk * g->nk) : NULL,
                box_mf ? malloc(sizeof(double) * nxk * g->nk) : NULL};
    double* k1 = malloc(sizeof(double) * N);
    double* k2 = malloc(sizeof(double) * N);
    double* t1 = malloc(sizeof(double) * N);
    double tau = prm->dt;
    int rc = 0;
    for (long st = 0; st < nsteps && rc == 0; ++st) {
        if (prm->scheme == 0) {
            /* Strang: A(tau/2); Heun on Theta with the potential frozen at the
             * sub-step start; A(tau/2). */
            if (or_advect_both(g, 0.5 * tau, f, t1)) { rc = -1; break; }
            or_symbols(&c, f);
            or_theta_all(&c, f, k1);
            for (long k = 0; k < N; ++k) t1[k] = f[k] + tau * k1[k];
            or_theta_all(&c, t1, k2);
            for (long k = 0; k < N; ++k) f[k] = f[k] + 0.5 * tau * (k1[k] + k2[k]);
            if (or_advect_both(g, 0.5 * tau, f, t1)) { rc = -1; break; }
        } else {
            /* Lawson predictor-corrector (Sec. 4.1):
             *   a = A_tau f, b = A_tau Theta[f], f~ = a + tau b,
             *   f+ = a + tau/2 Theta[f~] + tau/2 b. */
            or_symbols(&c, f);
            or_theta_all(&c, f, k1);
            if (or_advect_both(g, tau, f, t1)) { rc = -1; break; }   /* f  <- a */
            if (or_advect_both(g, tau, k1, t1)) { rc = -1; break; }  /* k1 <- b */
            for (long k = 0; k < N; ++k) t1[k] = f[k] + tau * k1[k]; /* f~ */
            or_symbols(&c, t1);
            or_theta_all(&c, t1, k2);
            for (long k = 0; k < N; ++k) f[k] = f[k] + 0.5 * tau * k2[k] + 0.5 * tau * k1[k];
        }
    }
    free(c.sig1); free(c.sig2); free(c.n1); free(c.n2); free(c.v);
    free(c.K1); free(c.K2);
    free(k1); free(k2); free(t1);
    return rc;
}

/* ------------------------------------------------------------------------ */
/* Observables (Sec. 2.2, Sec. 5 error metrics, Appendix B)                  */
/* ------------------------------------------------------------------------ */

/* scal = {mass, energy, l2}; n1[nx], n12[nx*nx], f1[nx*nk] (any may be NULL).
 * mass = sum dx^2 w w f; energy = sum dx^2 w w f (p1^2/2m + p2^2/2m + V(x1)
 * + V(x2) + V12(x1 - x2)); l2 = sum dx^2 w w f^2; n12 = sum_p w w f;
 * n1 = dx sum_i2 n12; f1(x1,p1) = dx sum_{i2,n2} w f (reduced Wigner function).*/
void or_observables(const or_grid* g, const double* f, const double* vext_x,
                    const double* v12_pair, double* scal, double* n1,
                    double* n12, double* f1)
{
    int nx = g->nx, nk = g->nk;
    double dx = or_dx(g);
    double* p = malloc(sizeof(double) * nk);
    double* w = malloc(sizeof(double) * nk);
    or_pnodes(g, p, w);
    double mass = 0.0, en = 0.0, l2 = 0.0;
    if (f1) for (long k = 0; k < (long)nx * nk; ++k) f1[k] = 0.0;
    if (n1) for (int i = 0; i < nx; ++i) n1[i] = 0.0;
    for (int i1 = 0; i1 < nx; ++i1)
        for (int i2 = 0; i2 < nx; ++i2) {
            const double* F = f + ((long)i1 * nx + i2) * nk * nk;
            double s0 = 0.0, sk = 0.0, s2 = 0.0;
            for (int a = 0; a < nk; ++a) {
                double row = 0.0;
                for (int b = 0; b < nk; ++b) {
                    double v = F[a * nk + b];
                    double ww = w[a] * w[b];
                    s0 += ww * v;
                    sk += ww * v * (p[a] * p[a] + p[b] * p[b]) / (2.0 * g->mass);
                    s2 += ww * v * v;
                    row += w[b] * v;
                }
                if (f1) f1[(long)i1 * nk + a] += dx * row;
            }
            double vpot = (vext_x ? vext_x[i1] + vext_x[i2] : 0.0) +
                          (v12_pair ? v12_pair[(long)i1 * nx + i2] : 0.0);
            mass += dx * dx * s0;
            en += dx * dx * (sk + vpot * s0);
            l2 += dx * dx * s2;
            if (n12) n12[(long)i1 * nx + i2] = s0;
            if (n1) n1[i1] += dx * s0;
        }
    if (scal) { scal[0] = mass; scal[1] = en; scal[2] = l2; }
    free(p);
    free(w);
}

/* Cyclic Jacobi eigenvalues of a real symmetric n x n matrix (destroys a). */
int or_jacobi_eigvals(int n, double* a, double* ev)
{
    for (int sweep = 0; sweep < 100; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < n; ++i)
            for (int j = i + 1; j < n; ++j) off += a[(long)i * n + j] * a[(long)i * n + j];
        if (off < 1e-30) break;
        for (int p = 0; p < n; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = a[(long)p * n + q];
                if (fabs(apq) < 1e-300) continue;
                double app = a[(long)p * n + p], aqq = a[(long)q * n + q];
                double th = (aqq - app) / (2.0 * apq);
                double t = (th >= 0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                double cs = 1.0 / sqrt(t * t + 1.0), sn = t * cs;
                for (int k = 0; k < n; ++k) {
                    double akp = a[(long)k * n + p], akq = a[(long)k * n + q];
                    a[(long)k * n + p] = cs * akp - sn * akq;
                    a[(long)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = a[(long)p * n + k], aqk = a[(long)q * n + k];
                    a[(long)p * n + k] = cs * apk - sn * aqk;
                    a[(long)q * n + k] = sn * apk + cs * aqk;
                }
            }
    }
    for (int i = 0; i < n; ++i) ev[i] = a[(long)i * n + i];
    return 0;
}

/* 1-RDM from the reduced Wigner function f1 (Appendix B, eq. DM_Wigner and the
 * discrete form that follows it):  with mid-point index mu and half-separation
 * nu,  rho1(x_{mu-nu}, x_{mu+nu}) = sum_n w_n f1(x_mu, p_n) e^{-i p_n 2 nu dx/hbar}.
 * Pairs (a, b) = (mu-nu, mu+nu) have equal parity, so rho1 is formed on the
 * even sub-lattice a, b in {0, 2, 4, ...}, where every mid-point is a grid node.
 * Occupations are the eigenvalues of (2 dx) rho1 (Hermitian), found by Jacobi on
 * the real embedding [[Re,-Im],[Im,Re]] (each eigenvalue appears twice), and are
 * normalised by their trace.  s_vn = -sum lam ln lam over lam > 1e-14.
 * evals[(nx+1)/2] ascending.  Returns the sub-lattice size. */
int or_rho1_entropy(const or_grid* g, const double* f1, double* evals, double* s_vn)
{
    int nx = g->nx, nk = g->nk, ns = (nx + 1) / 2, n2 = 2 * ns;
    double dx = or_dx(g);
    double* p = malloc(sizeof(double) * nk);
    double* w = malloc(sizeof(double) * nk);
    or_pnodes(g, p, w);
    double* E = calloc((size_t)n2 * n2, sizeof(double));
    for (int ia = 0; ia < ns; ++ia)
        for (int ib = 0; ib < ns; ++ib) {
            int a = 2 * ia, b = 2 * ib, mu = (a + b) / 2;
            const double* row = f1 + (long)mu * nk;
            double re = 0.0, im = 0.0;
            for (int n = 0; n < nk; ++n) {
                double ph = -p[n] * (b - a) * dx / g->hbar;
                re += w[n] * row[n] * cos(ph);
                im += w[n] * row[n] * sin(ph);
            }
            re *= 2.0 * dx;
            im *= 2.0 * dx;
            E[(long)ia * n2 + ib] = re;
            E[(long)(ia + ns) * n2 + ib + ns] = re;
            E[(long)(ia + ns) * n2 + ib] = im;
            E[(long)ia * n2 + ib + ns] = -im;
        }
    double* ev = malloc(sizeof(double) * n2);
    or_jacobi_eigvals(n2, E, ev);
    for (int i = 1; i < n2; ++i) {
        double t = ev[i];
        int j = i - 1;
        while (j >= 0 && ev[j] > t) { ev[j + 1] = ev[j]; --j; }
        ev[j + 1] = t;
    }
    double tr = 0.0;
    for (int i = 0; i < ns; ++i) { evals[i] = 0.5 * (ev[2 * i] + ev[2 * i + 1]); tr += evals[i]; }
    double s = 0.0;
    for (int i = 0; i < ns; ++i) {
        evals[i] /= tr;
        if (evals[i] > 1e-14) s -= evals[i] * log(evals[i]);
    }
    *s_vn = s;
    free(p); free(w); free(E); free(ev);
    return ns;
}
