// Internal declarations shared by the HIP translation units of libwig2.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "wig2.h"

namespace wig2 {

// Largest momentum-plane size handled by the fused Theta kernel (one plane in
// LDS: 128 x 129 FP64 = 129 KB of the 160 KB per CU).
constexpr int kMaxThetaNk = 128;

// ---------------------------------------------------------------------------
// Host-side symbol tables (tables.cpp).  All FP64.
// ---------------------------------------------------------------------------
struct GridInfo {
    int nx, nk, periodic, cells;
    double x_min, x_max, k_max, hbar, mass;
    double L() const { return x_max - x_min; }
    double dx() const { return periodic ? L() / nx : L() / (nx - 1); }
};

void host_nodes(const GridInfo& g, std::vector<double>& x, std::vector<double>& p,
                std::vector<double>& w);
// Periodic single-body symbol s[i][m] = (2/hbar) sig_m(x_i) from V at 2nk
// points y_j = x_min + j L/(2 nk).
void host_symbol_ext(const GridInfo& g, const std::vector<double>& v_y, std::vector<double>& s);
// Periodic pair kernel kap[l][m] = (2/hbar) Vhat_m sin(2 pi m l / nx), from
// V12 at r_j = -L/2 + j L/(2nk).
void host_pair_kernel(const GridInfo& g, const std::vector<double>& v12_r,
                      std::vector<double>& vhat, std::vector<double>& kap);
// Box single-body SEM matrices K[i][n][n'] from V at the x nodes.
void host_sem_matrix(const GridInfo& g, const std::vector<double>& v_x, std::vector<double>& K);
// Factors of that operator over the node distance d = i - j in [-(nx-1), nx-1]:
// E[(d + nx - 1)][n][s] = e^{2 i (p_n - d_s) d dx / hbar}, Q[(d + nx - 1)][k] =
// Q_k(-h d dx / hbar) (complex, re/im pairs), K = pref sum_j V_j Im(E Q).
void host_sem_factors(const GridInfo& g, std::vector<double>& E, std::vector<double>& Q, double& pref);
// Box two-body operator (Sec. 3.2.2): y-lattice spacing dy = pi hbar / |P|
// (|P| = 2 hbar k_max) and the real operands of its four matrix products
// (layouts in tables.cpp), from vs[l + nx - 1][d + nk - 1] = V12(l dx + d dy).
inline double sem12_dy(const GridInfo& g) { return 3.141592653589793238462643383279502884 / (2.0 * g.k_max); }
struct Sem12Tables {
    std::vector<double> wa, wb, wc, wd, dtab;
};
void host_sem12_tables(const GridInfo& g, const std::vector<double>& vs, Sem12Tables& t);
// Occupations of the trace-one 1-RDM built from f1 on the even sub-lattice.
double host_entropy(const GridInfo& g, const std::vector<double>& f1, std::vector<double>& occ);

// ---------------------------------------------------------------------------
// Kernel launchers.  T is double or float.
// ---------------------------------------------------------------------------

// One spline sweep along x_dim: out(x, p) = in(x - s p_dim / m, p).
// cells_per_p = s / (m dx); p_dev[nk] momentum nodes; work: state-sized scratch
// used only when the register-resident path does not cover (nx, shift).
// thomas_dev: Thomas multipliers for the box spline (nx entries).
// passes = 2 applies the same sweep twice in one launch (register-resident
// path only; hipErrorInvalidValue otherwise), bitwise equal to two launches.
// True when the register-resident sweep covers (nx, displacement); otherwise
// launch_advect needs the state-sized `work` array.
bool advect_in_registers(int nx, bool periodic, double max_cells);
template <typename T>
hipError_t launch_advect(const T* in, T* out, T* work, int nx, int nk, int dim, bool periodic,
                         double cells_per_p, double max_cells, const double* p_dev,
                         const double* thomas_dev, hipStream_t st, int passes = 1);

// Theta application on all nx*nx planes.
//   mode 0: out = Theta[u]
//   mode 1: out = u + tau/2 (v + Theta[u + tau v])   (out may equal u)
// sig1, sig2: [nx][nk] scaled single-body symbols (torus), band: largest m
// with a non-zero single-body symbol (nk-1 or more: dense).
// kap: [nx][nk] pair kernel (torus, NULL = no two-body term).
// ksem: [nx][nk][nk] single-body matrices (box; replaces sig1/sig2).
struct ThetaArgs {
    int nx, nk;
    const double* sig1;
    const double* sig2;
    int band;
    const double* kap;
    const double* ksem;
    int precision;  // WIG2_FP64 / WIG2_FP32 / WIG2_BF16X2
    const void* ksem_t;  // box, nk = 256: SEM matrices in the state's element type
    // box with a mean field: particle 2's SEM matrices (particle 1's are
    // ksem / ksem_t); NULL: both particles use ksem / ksem_t
    const double* ksem2 = nullptr;
    const void* ksem2_t = nullptr;
    // FFT path: device workspace of 3 nx (2 nk) doubles for the plane symbols
    double* fft_sym = nullptr;
};
template <typename T>
hipError_t launch_theta(const ThetaArgs& a, const T* u, const T* v, T* out, int mode, double tau,
                        hipStream_t st);
// One-pass Heun step of the general kernel (torus, nk = 32 .. 128, FP64 /
// FP32; theta_heun_general_ok tells where it applies):
// out = x + (tau/2)(Theta x + Theta (x + tau Theta x)); out may alias x.
bool theta_heun_general_ok(const ThetaArgs& a);
template <typename T>
hipError_t launch_theta_heun(const ThetaArgs& a, const T* x, T* out, double tau, hipStream_t st);

// Theta by 2-D FFT convolution of each momentum plane (theta_fft.hip):
// torus, nk in {16, 32, 48, 64, 96, 128}, FP64 / FP32, any single-body band.
// Same modes as launch_theta (0: out = Theta u; 1: out = u + tau/2 (v +
// Theta (u + tau v))).  Padded transform length: 2 nk rounded up to a
// multiple of the 64 lanes.
constexpr int fft_len(int nk) { return (2 * nk + 63) / 64 * 64; }
bool theta_fft_ok(const ThetaArgs& a);
template <typename T>
hipError_t launch_theta_fft(const ThetaArgs& a, const T* u, const T* v, T* out, int mode, double tau,
                            hipStream_t st);

// Box two-body operator (theta12_sem.hip).  Tables in the state's element
// type: wa (nk x 2nk), wb (2nk x 2nk), wc (2nk x 2nk), wd (2nk x nk), dtab
// ((2nx-1) x (2nk-1)).  pre: for the planes [plane0, plane0 + nplanes) of
// x = u + beta v (v may be NULL), the first three products into the
// workspaces wr, wh (2 nk^2 elements per plane each); post: the fourth,
// out = alpha Theta_12 x (accumulate = false) or out += alpha Theta_12 x.
struct Sem12Args {
    int nx, nk, ncu;
    const void *wa, *wb, *wc, *wd, *dtab;
};
bool sem12_nk_ok(int nk);
template <typename T>
hipError_t launch_sem12_pre(const Sem12Args& a, const T* u, const T* v, double beta, long plane0, long nplanes,
                            T* wr, T* wh, hipStream_t st);
template <typename T>
hipError_t launch_sem12_post(const Sem12Args& a, const T* wr, T* out, double alpha, bool accumulate, long plane0,
                             long nplanes, hipStream_t st);
// out[i] += acc[i], i < n
template <typename T>
hipError_t launch_sem12_add(const T* acc, T* out, long n, int ncu, hipStream_t st);

// Streaming Theta (theta_stream.hip) for the torus with a single-body band of
// at most 4 modes, FP64 or FP32, nk in {32, 48, 64, 96, 128}:
//   form 0: out = Theta[x]
//   form 1: out = x + tau Theta[x]
//   form 2: out = (y + x)/2 + (tau/2) Theta[x]
//   form 3: out = x + (tau/2)(Theta[x] + Theta[x + tau Theta[x]])  (Heun)
// out may alias x or y.
bool theta_stream_ok(const ThetaArgs& a);
constexpr int kStreamBand = 4;  // widest single-body band the streaming kernel does on the VALU
template <typename T>
hipError_t launch_theta_stream(const ThetaArgs& a, const T* x, const T* y, T* out, int form,
                               double tau, hipStream_t st);

// Split-BF16 streaming Theta (theta_stream_bf16.hip), FP32 state, torus,
// single-body band <= kStreamBand, nk in {32, 64, 96, 128}; forms as above.
bool theta_stream_bf16_ok(const ThetaArgs& a);
hipError_t launch_theta_stream_bf16(const ThetaArgs& a, const float* x, const float* y, float* out, int form,
                                    double tau, hipStream_t st);

// Panel Theta (theta_panel.hip) for box planes of nk = 256 (SEM matrices
// too large for the one-plane-in-LDS kernel), FP64, FP32 or split-BF16;
// forms as for the streaming kernel.  x and out must not be the same array
// for FP64 (two workgroups share a plane).
bool theta_panel_ok(const ThetaArgs& a);
template <typename T>
hipError_t launch_theta_panel(const ThetaArgs& a, const T* x, const T* y, T* out, int form,
                              double tau, hipStream_t st);

// Learned pair-increment surrogate (surrogate.hip): a 4-D separable
// convolutional network of kSurC channels (features of the pair term, one
// axis convolution per layer with a residual tanh, a linear output head),
// BF16 on the matrix cores, forward and backward.
constexpr int kSurC = 16;
struct SurScales {
    float in_scale;       // multiplies f_t in the features
    float out_scale;      // Delta = out_scale * y
    float inv_out_scale;
    float u_feat;         // pair-strength feature of the context
};
// One axis of the 4-D grid seen by a convolution: the axis (length La,
// stride Sa, periodic or zero outside), the lane axis that 16 consecutive
// points of a tile run along (length Ll, stride Sl), and the R positions of
// the two remaining coordinates, r -> (r / rdiv) rs_hi + (r % rdiv) rs_lo.
struct SurAxis {
    long Sa;
    int La, periodic;
    long Sl;
    int Ll;
    long R, rdiv, rs_hi, rs_lo;
};
size_t sur_conv_lds(int K);
size_t sur_dw_lds(int K);
long sur_tiles(const SurAxis& g);
// mode 0: training forward (hin -> tout = tanh(z), hout = hin + tout);
// 1: input gradient (dhin, tin -> dhout = dhin + conv^T(dhin (1 - tin^2)));
// 2: inference forward (hin -> hout).  wf: packed A fragments of the layer.
hipError_t launch_sur_conv(int mode, const SurAxis& g, int K, const unsigned short* hin, const float* dhin,
                           const unsigned short* tin, unsigned short* tout, unsigned short* hout, float* dhout,
                           const unsigned short* wf, const float* bias, int grid, hipStream_t st);
// Weight and bias gradient sums of one layer, part[grid][16 * 16 * K + 16].
hipError_t launch_sur_dw(const SurAxis& g, int K, const unsigned short* hin, const float* dhin,
                         const unsigned short* tin, float* part, int grid, hipStream_t st);
template <typename T>
hipError_t launch_sur_feat(const T* ft, int nx, int nk, const SurScales& sc, unsigned short* feat, hipStream_t st);
// mode 0: loss, dhL and head gradient sums; 1: loss only; 2: f += s_out y.
template <typename T>
hipError_t launch_sur_head(int mode, const unsigned short* hL, const unsigned short* feat, const T* delta, T* f,
                           long npts, const SurScales& sc, const float* head, float gscale, float* dhL, float* part,
                           float* lpart, hipStream_t st);
hipError_t launch_sur_reduce(const float* part, int nwg, int n, float scale, float* grad, hipStream_t st);
hipError_t launch_sur_adam(float* params, float* mom, float* var, const float* grad, long n, float lr, int step,
                           hipStream_t st);
hipError_t launch_sur_pack(const float* W, int K, int transposed, unsigned short* frag, hipStream_t st);
// d = a - b (when d != NULL) and per-workgroup max|a - b|, max|b| in part[2 nwg].
template <typename T>
hipError_t launch_diff_max(const T* a, const T* b, T* d, long n, float* part, int nwg, hipStream_t st);

// Per-plane moments: s0 = sum w w f, skin = sum w w f (p1^2+p2^2)/2m,
// s2 = sum w w f^2 (each [nx*nx]); rows[pl][n1] = sum_n2 w f (optional).
template <typename T>
hipError_t launch_plane_moments(const T* f, int nx, int nk, const double* p_dev,
                                const double* w_dev, double inv2m, double* s0, double* skin,
                                double* s2, double* rows, hipStream_t st);
// f1[i1][n1] = dx sum_i2 rows[i1*nx+i2][n1].
hipError_t launch_reduce_rows(const double* rows, int nx, int nk, double dx, double* f1,
                              hipStream_t st);
// Mean-field symbols from the plane sums s0 (torus):
//   n_1 = dx sum_i2 s0, n_2 = dx sum_i1 s0,
//   V_j = lambda dx sum V12pair n_j + xc terms,
//   sig_j[i][m] = sig_ext[i][m] + (2/hbar)(1/nx) sum_k V_j(x_k) sin(2 pi m (i-k)/nx), 2m < nx.
// If s0b != NULL the density is that of s0 + tau_b * s0b.
struct MeanFieldArgs {
    int nx, nk;
    double dx, lambda, hbar;
    int xc;
    double xc_n0, n_scale;
    const double* v12pair;  // [nx][nx]
    const double* sig_ext;  // [nx][nk], scaled by 2/hbar
    const double* sintab;   // [nk][nx] sin(2 pi m d / nx)
    double* dens;           // [2][nx] scratch
    double* veff;           // [2][nx] scratch
};
hipError_t launch_meanfield(const MeanFieldArgs& a, const double* s0, const double* s0b,
                            double tau_b, double* sig1, double* sig2, hipStream_t st);
// The density and effective-potential part alone (box contexts).
hipError_t launch_meanfield_potential(const MeanFieldArgs& a, const double* s0, const double* s0b, double tau_b,
                                      hipStream_t st);
// Box mean field: SEM matrices of V_ext + V_eff,j for both particles (FP64,
// plus FP32 copies when k1f is given) from veff [2][nx] and the factor
// tables E [(2nx-1)][nk][M] and Q [(2nx-1)][N] (complex, re/im pairs).
struct SemMfArgs {
    int nx, nk, nodes;
    double pref;
    const double* kext;  // [nx][nk][nk] SEM matrices of V_ext
    const double* veff;  // [2][nx]
    const double* E;
    const double* Q;
    double* k1;
    double* k2;
};
hipError_t launch_meanfield_sem(const SemMfArgs& a, float* k1f, float* k2f, hipStream_t st);

// ---------------------------------------------------------------------------
// Batched ensembles: one launch per phase walks a work list over all
// instances (batch.hip owns the host side).
// ---------------------------------------------------------------------------
struct BatchInst {
    long off;      // element offset of the instance in the state pools
    long tab_off;  // offset of its [nx][nk] symbol tables in the table pools
    int nx, nk;
    int p_off;     // offset of its momentum nodes in the node pool
    int band;
    int two_body;
    int pad;
    double cpp;    // half-step displacement per unit momentum, (dt/2)/(m dx)
    double tau;    // dt
};
struct AdvItem {   // 64 consecutive lines of one instance
    int inst;
    int pad;
    long line0;
};
struct ThItem {    // np consecutive planes of one instance
    int inst;
    int plane0;
    int np;
    int pad;
};
// Register-resident sizes the batched sweep supports.
bool batch_nx_ok(int nx);
bool batch_nk_ok(int nk);
// Largest number of planes of size nk one batched Theta workgroup holds
// (at most 4, 1024 threads and 160 KB of LDS).
int batch_theta_max_planes(int nk, int elem_bytes);
size_t batch_theta_lds(int nk, int np, int elem_bytes);

// Streaming one-pass Heun Theta over the items of one size class, in place on
// the state pool (instances with band <= kStreamBand, nk accepted by
// batch_stream_nk_ok; items are processed plane by plane).
bool batch_stream_nk_ok(int nk, int elem_bytes);
// Sizes for which the automatic choice takes the streaming kernel.
bool theta_stream_preferred(int nk, int elem_bytes);
template <typename T>
hipError_t launch_theta_stream_batch(T* pool, const BatchInst* insts, const ThItem* items, int nitems,
                                     const double* sig_pool, const double* kap_pool, int nk, int grid,
                                     hipStream_t st);

// One persistent launch over the items of one size class (all instances with
// this nx for the sweep, this nk for Theta).
template <typename T>
hipError_t launch_advect_batch(const T* in_pool, T* out_pool, const BatchInst* insts,
                               const AdvItem* items, int nitems, int dim, const double* p_pool,
                               int nx, int grid, hipStream_t st, int passes = 1);
template <typename T>
hipError_t launch_theta_batch(const T* u_pool, const T* v_pool, T* out_pool,
                              const BatchInst* insts, const ThItem* items, int nitems, int mode,
                              const double* sig_pool, const double* kap_pool, int nk, int planes,
                              int grid, hipStream_t st);

// Read-only view of one instance of a batched ensemble (batch.hip), for
// library-internal consumers such as the surrogate's trainer.
struct BatchView {
    GridInfo g;
    wig2_params prm;
    int elem;
    const void* f;        // instance state in the pool
    const double* sig;    // [nx][nk] single-body symbol
    const double* kap;    // [nx][nk] pair kernel
    int band, two_body;
    const std::vector<double>* vext_x;
    const std::vector<double>* v12pair;
    bool has_pot, has_state;
    hipStream_t st;
};
int batch_count(const wig2_batch* b);
bool batch_view(const wig2_batch* b, int i, BatchView& v);

}  // namespace wig2
