// Host-side FP64 tables of the method: grid nodes, Fourier symbols of the
// pseudo-difference operators, the spectral-element single-body matrices and
// the 1-RDM entropy.  Built once per wig2_set_potentials (or per observable
// call for the entropy); never on the time-step path.
#include <cmath>
#include <complex>
#include <thread>
#include <vector>

#include "common.h"

namespace wig2 {

namespace {
constexpr double kPi = 3.141592653589793238462643383279502884;
typedef std::complex<double> cplx;

// Chebyshev-Gauss nodes of one cell in increasing order, eta_k = -cos(theta_k).
void cheb_nodes(int N, std::vector<double>& eta, std::vector<double>& bw)
{
    eta.resize(N);
    bw.resize(N);
    for (int k = 0; k < N; ++k) {
        const double th = (2.0 * k + 1.0) * kPi / (2.0 * N);
        eta[k] = -std::cos(th);
        bw[k] = ((k & 1) ? -1.0 : 1.0) * std::sin(th);  // barycentric weights
    }
}

// Lagrange cardinal polynomial ell_k(x) on the nodes (barycentric form).
double cardinal(const std::vector<double>& eta, const std::vector<double>& bw, int k, double x)
{
    double den = 0.0;
    for (size_t j = 0; j < eta.size(); ++j) {
        const double d = x - eta[j];
        if (std::fabs(d) < 1e-300) return (int)j == k ? 1.0 : 0.0;
        den += bw[j] / d;
    }
    return (bw[k] / (x - eta[k])) / den;
}

// Gauss-Legendre rule on [-1, 1] (Golub-Welsch free: Newton on P_q with the
// asymptotic start values).
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w)
{
    x.resize(q);
    w.resize(q);
    for (int i = 0; i < (q + 1) / 2; ++i) {
        double z = std::cos(kPi * (4.0 * i + 3.0) / (4.0 * q + 2.0));
        double dp = 1.0;
        for (int it = 0; it < 60; ++it) {
            double p0 = 1.0, p1 = z;
            for (int k = 2; k <= q; ++k) {
                const double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            dp = q * (p0 - z * p1) / (1.0 - z * z);
            const double step = p1 / dp;
            z -= step;
            if (std::fabs(step) < 5e-17) break;
        }
        x[i] = -z;
        x[q - 1 - i] = z;
        w[i] = w[q - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}
}  // namespace

void host_nodes(const GridInfo& g, std::vector<double>& x, std::vector<double>& p,
                std::vector<double>& w)
{
    x.resize(g.nx);
    p.resize(g.nk);
    w.resize(g.nk);
    const double dx = g.dx();
    for (int i = 0; i < g.nx; ++i) x[i] = g.x_min + dx * i;
    if (g.periodic) {
        const double dp = g.hbar * kPi / g.L();
        for (int n = 0; n < g.nk; ++n) {
            p[n] = dp * (n - g.nk / 2);
            w[n] = dp;
        }
        return;
    }
    // Box: cells of width h on [-hbar k_max, hbar k_max]; per cell the weights
    // integrate the Chebyshev interpolant: w_k = (h/2) int ell_k, with
    // int ell_k = sum_l c_l T_l(eta_k) int T_l, int T_l = 2/(1 - l^2) (l even).
    const int M = g.cells, N = g.nk / g.cells;
    const double pm = g.hbar * g.k_max, h = 2.0 * pm / M;
    std::vector<double> eta, bw;
    cheb_nodes(N, eta, bw);
    for (int s = 0; s < M; ++s) {
        const double mid = -pm + h * (s + 0.5);
        for (int k = 0; k < N; ++k) {
            double iw = 0.0;
            const double th = (2.0 * k + 1.0) * kPi / (2.0 * N);
            for (int l = 0; l < N; l += 2) {
                const double Tl = std::cos(l * (kPi - th));  // T_l(-cos th)
                iw += (l == 0 ? 1.0 : 2.0) / N * Tl * 2.0 / (1.0 - (double)l * l);
            }
            p[s * N + k] = mid + 0.5 * h * eta[k];
            w[s * N + k] = 0.5 * h * iw;
        }
    }
}

void host_symbol_ext(const GridInfo& g, const std::vector<double>& v_y, std::vector<double>& s)
{
    const int nx = g.nx, nk = g.nk, ny = 2 * nk;
    const double L = g.L(), dx = g.dx();
    // Vhat_m = (1/2nk) sum_j V(y_j) e^{+2 pi i m y_j / L}
    std::vector<cplx> vh(nk);
    for (int m = 0; m < nk; ++m) {
        cplx acc(0.0, 0.0);
        for (int j = 0; j < ny; ++j) {
            const double y = g.x_min + L * j / ny;
            acc += v_y[j] * std::polar(1.0, 2.0 * kPi * m * y / L);
        }
        vh[m] = acc / (double)ny;
    }
    s.assign((size_t)nx * nk, 0.0);
    for (int i = 0; i < nx; ++i) {
        const double x = g.x_min + dx * i;
        for (int m = 1; m < nk; ++m) {
            const cplx e = vh[m] * std::polar(1.0, -2.0 * kPi * m * x / L);
            s[(size_t)i * nk + m] = (2.0 / g.hbar) * (-e.imag());
        }
    }
}

void host_pair_kernel(const GridInfo& g, const std::vector<double>& v12_r,
                      std::vector<double>& vhat, std::vector<double>& kap)
{
    const int nx = g.nx, nk = g.nk, ny = 2 * nk;
    const double L = g.L();
    vhat.assign(nk, 0.0);
    for (int m = 0; m < nk; ++m) {
        cplx acc(0.0, 0.0);
        for (int j = 0; j < ny; ++j) {
            const double r = -0.5 * L + L * j / ny;
            acc += v12_r[j] * std::polar(1.0, 2.0 * kPi * m * r / L);
        }
        vhat[m] = acc.real() / ny;  // even V12: the imaginary part is rounding
    }
    kap.assign((size_t)nx * nk, 0.0);
    for (int l = 0; l < nx; ++l)
        for (int m = 1; m < nk; ++m)
            kap[(size_t)l * nk + m] = (2.0 / g.hbar) * vhat[m] * std::sin(2.0 * kPi * m * l / nx);
}

// Box single-body operator (Sec. 3.2.1).  With the first-principles i/hbar
// and the x-grid sum for the Fourier transform of V,
//   V_W(x, q) = (2 dx / (pi hbar^2)) sum_j V(x_j) sin(2 q (x - x_j) / hbar),
// and the p'-integral over cell s of the cell interpolant of f,
//   int_{P_s} V_W(x_i, p_n - p') f(p') dp'
//     = sum_k f(p_{s,k}) (2 dx/(pi hbar^2)) (h/2) sum_j V(x_j)
//       Im[ e^{2 i (p_n - d_s) z / hbar} Q_k(-h z / hbar) ],  z = x_i - x_j,
// where Q_k(zeta) = int_{-1}^{1} e^{i zeta eta} ell_k(eta) d eta is the
// oscillatory integral of the cell's Lagrange cardinal function (the
// Chebyshev combination of the paper's O_l).  Q_k by Gauss-Legendre.
void host_sem_matrix(const GridInfo& g, const std::vector<double>& v_x, std::vector<double>& K)
{
    const int nx = g.nx, nk = g.nk, M = g.cells, N = nk / M;
    const double hb = g.hbar, dx = g.dx();
    const double pm = hb * g.k_max, h = 2.0 * pm / M;
    std::vector<double> x, p, w, eta, bw;
    host_nodes(g, x, p, w);
    cheb_nodes(N, eta, bw);
    // Q[d][k] for z = d dx, d in [-(nx-1), nx-1]
    const int nd = 2 * nx - 1;
    std::vector<cplx> Q((size_t)nd * N);
    for (int d = -(nx - 1); d <= nx - 1; ++d) {
        const double zeta = -h * d * dx / hb;
        const int q = std::max(48, (int)std::ceil(std::fabs(zeta)) + 2 * N + 40);
        std::vector<double> gx, gw;
        gauss_legendre(q, gx, gw);
        for (int k = 0; k < N; ++k) {
            cplx acc(0.0, 0.0);
            for (int t = 0; t < q; ++t)
                acc += gw[t] * cardinal(eta, bw, k, gx[t]) * std::polar(1.0, zeta * gx[t]);
            Q[(size_t)(d + nx - 1) * N + k] = acc;
        }
    }
    K.assign((size_t)nx * nk * nk, 0.0);
    const double pref = 2.0 * dx / (kPi * hb * hb) * 0.5 * h;
    auto work = [&](int i0, int i1) {
        for (int i = i0; i < i1; ++i)
            for (int n = 0; n < nk; ++n)
                for (int s = 0; s < M; ++s) {
                    const double ds = -pm + h * (s + 0.5);
                    double* row = &K[((size_t)i * nk + n) * nk + (size_t)s * N];
                    for (int j = 0; j < nx; ++j) {
                        if (v_x[j] == 0.0) continue;
                        const double z = (i - j) * dx;
                        const cplx e = std::polar(1.0, 2.0 * (p[n] - ds) * z / hb);
                        const cplx* q = &Q[(size_t)(i - j + nx - 1) * N];
                        for (int k = 0; k < N; ++k) row[k] += v_x[j] * (e * q[k]).imag();
                    }
                    for (int k = 0; k < N; ++k) row[k] *= pref;
                }
    };
    unsigned nt = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
    std::vector<std::thread> th;
    const int chunk = (nx + (int)nt - 1) / (int)nt;
    for (unsigned t = 0; t < nt; ++t) {
        const int a = (int)t * chunk, b = std::min(nx, a + chunk);
        if (a < b) th.emplace_back(work, a, b);
    }
    for (auto& t : th) t.join();
}

// Box two-body operator (Sec. 3.2.2), host tables.  y-lattice: the nk
// midpoints y_j = (j + 1/2 - nk/2) dy, dy = pi hbar / |P| (|P| = 2 hbar k_max,
// the sums over y are then |P|-periodic in p).  Complex
//   G[y][n] = int_{P_s} e^{2 i p y / hbar} ell_n(p) dp
//           = (h/2) e^{2 i d_s y / hbar} Q_k(h y / hbar)      (n = s N + k)
//   B[n][y] = e^{-2 i p_n y / hbar}
// so that G F G^T is the y-transform of the cell-wise interpolant of a plane F
// and Im(B H B^T) the back-transform; the real operands of the four matrix
// products (layouts in theta12_sem.hip):
//   WA[k][j]      = Re G[j][k],  WA[k][ny + j] = Im G[j][k]            (nk x 2ny)
//   WB[y][2k]     = Re G[y][k],  WB[y][2k+1] = -Im G[y][k],
//   WB[ny+y][2k]  = Im G[y][k],  WB[ny+y][2k+1] = Re G[y][k]          (2ny x 2nk)
//   WC[2n][y]     = Re B[n][y],  WC[2n][ny+y] = -Im B[n][y],
//   WC[2n+1][y]   = Im B[n][y],  WC[2n+1][ny+y] = Re B[n][y]          (2nk x 2ny)
//   WD[y][n]      = Im B[n][y],  WD[ny+y][n] = Re B[n][y]              (2ny x nk)
// and the potential difference, with the constant of the y-sum folded in,
//   D[l + nx - 1][d + ny - 1] = (dy^2/(pi^2 hbar^3)) (V12(l dx + d dy) - V12(l dx - d dy))
// from vs[l + nx - 1][d + ny - 1] = V12(l dx + d dy).
void host_sem12_tables(const GridInfo& g, const std::vector<double>& vs, Sem12Tables& t)
{
    const int nx = g.nx, nk = g.nk, ny = g.nk, M = g.cells, N = nk / M;
    const double hb = g.hbar, pm = hb * g.k_max, h = 2.0 * pm / M;
    const double dy = sem12_dy(g);
    std::vector<double> x, p, w, eta, bw;
    host_nodes(g, x, p, w);
    cheb_nodes(N, eta, bw);
    std::vector<cplx> G((size_t)ny * nk), Bm((size_t)nk * ny);
    for (int j = 0; j < ny; ++j) {
        const double y = (j + 0.5 - 0.5 * ny) * dy;
        const double zeta = h * y / hb;
        const int q = std::max(48, (int)std::ceil(std::fabs(zeta)) + 2 * N + 40);
        std::vector<double> gx, gw;
        gauss_legendre(q, gx, gw);
        for (int k = 0; k < N; ++k) {
            cplx Qk(0.0, 0.0);
            for (int tq = 0; tq < q; ++tq) Qk += gw[tq] * cardinal(eta, bw, k, gx[tq]) * std::polar(1.0, zeta * gx[tq]);
            for (int s = 0; s < M; ++s) {
                const double ds = -pm + h * (s + 0.5);
                G[(size_t)j * nk + s * N + k] = 0.5 * h * std::polar(1.0, 2.0 * ds * y / hb) * Qk;
            }
        }
        for (int n = 0; n < nk; ++n) Bm[(size_t)n * ny + j] = std::polar(1.0, -2.0 * p[n] * y / hb);
    }
    t.wa.assign((size_t)nk * 2 * ny, 0.0);
    t.wb.assign((size_t)2 * ny * 2 * nk, 0.0);
    t.wc.assign((size_t)2 * nk * 2 * ny, 0.0);
    t.wd.assign((size_t)2 * ny * nk, 0.0);
    for (int j = 0; j < ny; ++j)
        for (int k = 0; k < nk; ++k) {
            const cplx gv = G[(size_t)j * nk + k];
            t.wa[(size_t)k * 2 * ny + j] = gv.real();
            t.wa[(size_t)k * 2 * ny + ny + j] = gv.imag();
            t.wb[(size_t)j * 2 * nk + 2 * k] = gv.real();
            t.wb[(size_t)j * 2 * nk + 2 * k + 1] = -gv.imag();
            t.wb[(size_t)(ny + j) * 2 * nk + 2 * k] = gv.imag();
            t.wb[(size_t)(ny + j) * 2 * nk + 2 * k + 1] = gv.real();
        }
    for (int n = 0; n < nk; ++n)
        for (int j = 0; j < ny; ++j) {
            const cplx bv = Bm[(size_t)n * ny + j];
            t.wc[(size_t)2 * n * 2 * ny + j] = bv.real();
            t.wc[(size_t)2 * n * 2 * ny + ny + j] = -bv.imag();
            t.wc[(size_t)(2 * n + 1) * 2 * ny + j] = bv.imag();
            t.wc[(size_t)(2 * n + 1) * 2 * ny + ny + j] = bv.real();
            t.wd[(size_t)j * nk + n] = bv.imag();
            t.wd[(size_t)(ny + j) * nk + n] = bv.real();
        }
    const double c = dy * dy / (kPi * kPi * hb * hb * hb);
    const int nd = 2 * ny - 1;
    t.dtab.assign((size_t)(2 * nx - 1) * nd, 0.0);
    for (int l = 0; l < 2 * nx - 1; ++l)
        for (int d = -(ny - 1); d <= ny - 1; ++d)
            t.dtab[(size_t)l * nd + d + ny - 1] = c * (vs[(size_t)l * nd + d + ny - 1] - vs[(size_t)l * nd - d + ny - 1]);
}

// The factors of host_sem_matrix's kernel over the node distance, for the
// mean field's matrices rebuilt on the device.
void host_sem_factors(const GridInfo& g, std::vector<double>& E, std::vector<double>& Q, double& pref)
{
    const int nx = g.nx, nk = g.nk, M = g.cells, N = nk / M;
    const double hb = g.hbar, dx = g.dx();
    const double pm = hb * g.k_max, h = 2.0 * pm / M;
    std::vector<double> x, p, w, eta, bw;
    host_nodes(g, x, p, w);
    cheb_nodes(N, eta, bw);
    const int nd = 2 * nx - 1;
    Q.assign((size_t)2 * nd * N, 0.0);
    E.assign((size_t)2 * nd * nk * M, 0.0);
    for (int d = -(nx - 1); d <= nx - 1; ++d) {
        const double zeta = -h * d * dx / hb;
        const int q = std::max(48, (int)std::ceil(std::fabs(zeta)) + 2 * N + 40);
        std::vector<double> gx, gw;
        gauss_legendre(q, gx, gw);
        const size_t di = (size_t)(d + nx - 1);
        for (int k = 0; k < N; ++k) {
            cplx acc(0.0, 0.0);
            for (int t = 0; t < q; ++t) acc += gw[t] * cardinal(eta, bw, k, gx[t]) * std::polar(1.0, zeta * gx[t]);
            Q[2 * (di * N + k)] = acc.real();
            Q[2 * (di * N + k) + 1] = acc.imag();
        }
        for (int n = 0; n < nk; ++n)
            for (int s = 0; s < M; ++s) {
                const double ds = -pm + h * (s + 0.5);
                const cplx e = std::polar(1.0, 2.0 * (p[n] - ds) * d * dx / hb);
                E[2 * ((di * nk + n) * M + s)] = e.real();
                E[2 * ((di * nk + n) * M + s) + 1] = e.imag();
            }
    }
    pref = 2.0 * dx / (kPi * hb * hb) * 0.5 * h;
}

// 1-RDM from the reduced Wigner function (Appendix B):
//   rho1(x_{mu-nu}, x_{mu+nu}) = sum_n w_n f1(x_mu, p_n) e^{-2 i p_n nu dx / hbar},
// on the even sub-lattice (all mid-points on the grid).  Eigenvalues of the
// Hermitian (2 dx) rho1 by complex Jacobi rotations; occupations normalised to
// trace one; returns -sum lam ln lam over lam > 1e-14.
double host_entropy(const GridInfo& g, const std::vector<double>& f1, std::vector<double>& occ)
{
    const int nx = g.nx, nk = g.nk, ns = (nx + 1) / 2;
    std::vector<double> x, p, w;
    host_nodes(g, x, p, w);
    const double dx = g.dx();
    std::vector<cplx> A((size_t)ns * ns);
    for (int a = 0; a < ns; ++a)
        for (int b = 0; b < ns; ++b) {
            const int mu = a + b;  // (2a + 2b)/2
            cplx s(0.0, 0.0);
            for (int n = 0; n < nk; ++n)
                s += w[n] * f1[(size_t)mu * nk + n] *
                     std::polar(1.0, -p[n] * (2.0 * (b - a)) * dx / g.hbar);
            A[(size_t)a * ns + b] = 2.0 * dx * s;
        }
    // cyclic complex Jacobi
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = 0.0;
        for (int i = 0; i < ns; ++i)
            for (int j = i + 1; j < ns; ++j) off += std::norm(A[(size_t)i * ns + j]);
        if (off < 1e-32) break;
        for (int pq = 0; pq < ns; ++pq)
            for (int qq = pq + 1; qq < ns; ++qq) {
                const cplx apq = A[(size_t)pq * ns + qq];
                const double mag = std::abs(apq);
                if (mag < 1e-300) continue;
                const double app = A[(size_t)pq * ns + pq].real(), aqq = A[(size_t)qq * ns + qq].real();
                const cplx ph = apq / mag;  // e^{i phi}
                const double tau = (aqq - app) / (2.0 * mag);
                const double t = (tau >= 0 ? 1.0 : -1.0) / (std::fabs(tau) + std::sqrt(1.0 + tau * tau));
                const double c = 1.0 / std::sqrt(1.0 + t * t), sn = t * c;
                // columns: A <- A R, R = [[c, s e^{i phi}], [-s e^{-i phi}, c]] acting on (p, q)
                for (int k = 0; k < ns; ++k) {
                    const cplx akp = A[(size_t)k * ns + pq], akq = A[(size_t)k * ns + qq];
                    A[(size_t)k * ns + pq] = c * akp - sn * std::conj(ph) * akq;
                    A[(size_t)k * ns + qq] = sn * ph * akp + c * akq;
                }
                for (int k = 0; k < ns; ++k) {
                    const cplx apk = A[(size_t)pq * ns + k], aqk = A[(size_t)qq * ns + k];
                    A[(size_t)pq * ns + k] = c * apk - sn * ph * aqk;
                    A[(size_t)qq * ns + k] = sn * std::conj(ph) * apk + c * aqk;
                }
            }
    }
    occ.resize(ns);
    double tr = 0.0;
    for (int i = 0; i < ns; ++i) {
        occ[i] = A[(size_t)i * ns + i].real();
        tr += occ[i];
    }
    double s = 0.0;
    for (int i = 0; i < ns; ++i) {
        occ[i] /= tr;
        if (occ[i] > 1e-14) s -= occ[i] * std::log(occ[i]);
    }
    return s;
}

}  // namespace wig2
