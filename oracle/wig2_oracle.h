/*
 * wig2_oracle.h -- plain FP64 CPU reference ("oracle") for one time step of the
 * two-body Wigner equation of Liang & Xiong, arXiv:2511.11354.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library includes, links or
 * calls this code; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or helper with the HIP
 * path.  Every routine is a direct, unblocked transcription of the definition
 * it cites, in FP64, with no BLAS and no FFT.
 *
 * Layout of a 4-D state: f[((i1*nx + i2)*nk + n1)*nk + n2]  (n2 fastest).
 */
#ifndef WIG2_ORACLE_H
#define WIG2_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int nx, nk;        /* points per x-dimension, per p-dimension               */
    int periodic;      /* 1: torus [x_min,x_max); 0: box with natural spline     */
    int cells;         /* non-periodic: SEM cells per p-dimension                */
    double x_min, x_max;
    double k_max;      /* non-periodic: p-box is [-hbar*k_max, hbar*k_max]       */
    double hbar, mass;
} or_grid;

typedef struct {
    double dt;
    int scheme;        /* 0: Strang (A/2, Heun on Theta, A/2); 1: Lawson PC     */
    double lambda;     /* mean-field Hartree weight                              */
    int xc;            /* 1: add the Hedin-Lundqvist exchange-correlation term   */
    double xc_n0, n_scale;
    int two_body;      /* 1: include Theta_V12                                   */
    int hartree;       /* 0: Hartree by convolution with V12 (Sec. 2.3); 1: the
                          neutralised Poisson potential (Sec. 3.1.1 example)   */
} or_params;

typedef struct {
    const double* sig_ext;  /* periodic: [nx][nk] single-body symbol of V_ext   */
    const double* vhat12;   /* periodic: [nk] Fourier modes of V12                */
    const double* K;        /* non-periodic: [nx][nk][nk] SEM single-body matrix  */
    const double* v12_pair; /* [nx][nx] V12(x_i1 - x_i2) (minimum image if torus) */
    const double* v12_sem;  /* non-periodic: [2nx-1][2nk-1] V12(l dx + d dy) for the
                               two-body SEM operator, or NULL (no pair term)       */
} or_tables;

int    or_num_threads(void);
void   or_set_threads(int n);
double or_dx(const or_grid* g);
void   or_xnodes(const or_grid* g, double* x);
void   or_pnodes(const or_grid* g, double* p, double* w);

void or_sigma_ext(const or_grid* g, const double* v_y, double* sig);
void or_vhat12(const or_grid* g, const double* v12_r, double* vhat);
void or_sigma_hxc(const or_grid* g, const double* v_x, double* sig);
void or_veff_hxc(const or_grid* g, const or_params* prm, const double* v12_pair,
                 const double* n, double* v);
void or_densities(const or_grid* g, const double* f, double* n1, double* n2);
void or_hartree_poisson(const or_grid* g, const double* n, double* v);
void or_hartree_padded(const or_grid* g, const double* v12_pad, const double* n, double* v);

void or_theta_periodic(const or_grid* g, const double* sig1, const double* sig2,
                       const double* vhat12, int two_body,
                       long plane0, long nplanes, const double* f, double* out);
void or_theta_dense(const or_grid* g, const double* K1, const double* K2,
                    long plane0, long nplanes, const double* f, double* out);
void or_sem_kernel(const or_grid* g, const double* v_x, double* K);
double or_sem12_dy(const or_grid* g);
void or_theta12_sem(const or_grid* g, const double* v12_tab, long plane0, long nplanes,
                    const double* f, double* out);

int  or_advect(const or_grid* g, int dim, double s, long line0, long nlines,
               const double* f, double* out);

int  or_step(const or_grid* g, const or_params* prm, const or_tables* tb,
             double* f, long nsteps);

void or_observables(const or_grid* g, const double* f, const double* vext_x,
                    const double* v12_pair, double* scal, double* n1,
                    double* n12, double* f1);
int  or_rho1_entropy(const or_grid* g, const double* f1, double* evals /*(nx+1)/2*/,
                     double* s_vn);
int  or_jacobi_eigvals(int n, double* a, double* ev);

#ifdef __cplusplus
}
#endif
#endif
