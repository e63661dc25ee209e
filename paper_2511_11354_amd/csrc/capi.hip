// C ABI of libwig2 (declared in include/wig2.h): context, tables, the step
// schedule and the observables.  All time-stepping work runs in the HIP
// kernels of advect.hip / theta.hip / reduce.hip on the context stream.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "common.h"

using namespace wig2;

// Scratch of the allocation-free sweep (wig2_advect_noalloc): the spline
// coefficients of the general sweep, laid out like the state, for states of
// at most kNoAllocScratchBytes.  Every device the library runs on holds its
// own copy until the process ends.  Host code never passes `scratch` itself
// to a kernel: it passes the device address that hipGetSymbolAddress returns
// for the current device (noalloc_scratch).
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on `device` (the current device), resolved
// once per device.  Called from wig2_create.
hipError_t resolve_noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (g_scratch_ptr[device]) return hipSuccess;
    void* ptr = nullptr;
    hipError_t e = hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[device] = ptr;
    return hipSuccess;
}

void* noalloc_scratch(int device)
{
    if (device < 0 || device >= kMaxDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_ptr[device];
}
}  // namespace

struct wig2_ctx {
    GridInfo g{};
    wig2_params prm{};
    int device = 0;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int elem = 8;
    long npts = 0;
    void* f = nullptr;       // the state: f_own, or a caller-owned buffer (wig2_bind_state)
    void* f_own = nullptr;   // state buffer allocated by the context
    void* k1 = nullptr;
    void* tmp = nullptr;
    void* work = nullptr;  // lazily allocated advection scratch
    double *p_d = nullptr, *w_d = nullptr, *thomas_d = nullptr;
    double *sig_ext_d = nullptr, *sig1_d = nullptr, *sig2_d = nullptr, *kap_d = nullptr;
    double *ksem_d = nullptr, *v12pair_d = nullptr, *sintab_d = nullptr;
    float* ksem_f = nullptr;  // FP32 copy of the SEM matrices (nk = 256, FP32 / BF16X2)
    double *mf_dens_d = nullptr, *mf_veff_d = nullptr;
    double *s0_d = nullptr, *s0b_d = nullptr, *skin_d = nullptr, *s2_d = nullptr;
    double *rows_d = nullptr, *f1_d = nullptr;
    int band = 0;
    int theta_path = WIG2_THETA_AUTO;
    bool two_body = false, meanfield = false;
    bool fuse_sweeps = true;  // Strang: consecutive x1 half-sweeps in one launch
    std::vector<double> x, p, w, vext_x, v12pair;
    double pmax = 0.0;
    bool has_state = false, has_pot = false;
    int64_t nstep = 0;
    double t = 0.0;
    std::string err;
    // per-kernel-class HIP event timing (wig2_profile)
    bool prof = false;
    std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> prof_ev;
    std::vector<hipEvent_t> ev_pool;
    double prof_ms[WIG2_PROF_N] = {};
    int64_t prof_cnt[WIG2_PROF_N] = {};
    // learned pair-increment surrogate (wig2_surrogate_*)
    bool no_pair = false;            // steps leave out Theta[V12]
    void* ft = nullptr;              // block-start state
    void* fs = nullptr;              // second block result
    const wig2_surrogate* sur = nullptr;
    double sur_tol = 0.0;
    int sur_every = 0, sur_since = 0;
    int64_t sur_blocks = 0, sur_fallbacks = 0, sur_checks = 0;
    double sur_last_err = -1.0;
    bool sur_ref_ok = false;
    double sur_mref = 0.0, sur_eref = 0.0;
};

struct wig2_surrogate {
    int device = 0;
    wig2_train_cfg cfg{};
    float* params = nullptr;
    float* mom = nullptr;
    float* var = nullptr;
    unsigned short* pbf = nullptr;
    float* partial = nullptr;  // [batch / 256][kSurP]
    float* lpart = nullptr;    // loss sums per workgroup, one epoch
    long lpart_cap = 0;
    float* grad = nullptr;     // [kSurP]
    float* maxpart = nullptr;  // [2 * kMaxParts]
    wig2::SurScales sc{1.f, 1.f, 1.f, 0.f};
    bool scaled = false;
    double dt = 0.0;
    int64_t updates = 0, samples = 0;
    double train_loss = -1.0, eval_loss = -1.0;
    std::string err;
};

namespace {

hipEvent_t pool_event(wig2_ctx* c)
{
    if (!c->ev_pool.empty()) {
        hipEvent_t e = c->ev_pool.back();
        c->ev_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Wrap one launch of kernel class k in a pair of events when profiling.
template <typename F>
hipError_t timed(wig2_ctx* c, int k, F&& launch)
{
    if (!c->prof) return launch();
    hipEvent_t a = pool_event(c), b = pool_event(c);
    if (!a || !b) return launch();
    hipEventRecord(a, c->st);
    hipError_t e = launch();
    hipEventRecord(b, c->st);
    c->prof_ev.push_back({k, {a, b}});
    return e;
}

int fail(wig2_ctx* c, int code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

#define HIPCHK(ctx, call)                                                                   \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(ctx, e_ == hipErrorOutOfMemory ? WIG2_ENOMEM : WIG2_EDEVICE,        \
                        std::string(#call) + ": " + hipGetErrorString(e_));                 \
    } while (0)

bool isfin(double v) { return std::isfinite(v); }

template <typename T>
int dev_alloc(wig2_ctx* c, T** p, size_t n)
{
    if (n == 0) n = 1;
    hipError_t e = hipMalloc((void**)p, n * sizeof(T));
    if (e != hipSuccess) return fail(c, WIG2_ENOMEM, std::string("hipMalloc: ") + hipGetErrorString(e));
    return 0;
}

int upload(wig2_ctx* c, double* d, const std::vector<double>& h)
{
    HIPCHK(c, hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    return 0;
}

bool theta_nk_ok(int nk) { return nk == 16 || nk == 32 || nk == 48 || nk == 64 || nk == 96 || nk == 128; }
// Box planes of this size take the panel Theta kernel.
constexpr int kPanelThetaNk = 256;

// ---- step building blocks -------------------------------------------------

template <typename T>
hipError_t advect(wig2_ctx* c, int dim, double s, const T* in, T* out)
{
    const double cpp = s / (c->g.mass * c->g.dx());
    const double maxc = std::fabs(cpp) * c->pmax;
    T* wk = static_cast<T*>(c->work);
    return launch_advect<T>(in, out, wk, c->g.nx, c->g.nk, dim, c->g.periodic != 0, cpp, maxc, c->p_d,
                            c->thomas_d, c->st);
}

template <typename T>
hipError_t moments(wig2_ctx* c, const T* f, double* s0, double* skin, double* s2, double* rows)
{
    return launch_plane_moments<T>(f, c->g.nx, c->g.nk, c->p_d, c->w_d, 0.5 / c->g.mass, s0, skin, s2,
                                   rows, c->st);
}

MeanFieldArgs mf_args(wig2_ctx* c)
{
    MeanFieldArgs a;
    a.nx = c->g.nx;
    a.nk = c->g.nk;
    a.dx = c->g.dx();
    a.lambda = c->prm.meanfield_lambda;
    a.hbar = c->g.hbar;
    a.xc = c->prm.xc;
    a.xc_n0 = c->prm.xc_n0;
    a.n_scale = c->prm.n_scale;
    a.v12pair = c->v12pair_d;
    a.sig_ext = c->sig_ext_d;
    a.sintab = c->sintab_d;
    a.dens = c->mf_dens_d;
    a.veff = c->mf_veff_d;
    return a;
}

ThetaArgs theta_args(wig2_ctx* c)
{
    ThetaArgs a;
    a.nx = c->g.nx;
    a.nk = c->g.nk;
    a.sig1 = c->meanfield ? c->sig1_d : c->sig_ext_d;
    a.sig2 = c->meanfield ? c->sig2_d : c->sig_ext_d;
    a.band = c->meanfield ? c->g.nk : c->band;
    a.kap = (c->two_body && !c->no_pair) ? c->kap_d : nullptr;
    a.ksem = c->g.periodic ? nullptr : c->ksem_d;
    a.precision = c->prm.precision;
    a.ksem_t = nullptr;
    if (!c->g.periodic && c->g.nk == kPanelThetaNk)
        a.ksem_t = c->elem == 8 ? (const void*)c->ksem_d : (const void*)c->ksem_f;
    return a;
}

template <typename T>
hipError_t theta(wig2_ctx* c, const T* u, const T* v, T* out, int mode, double tau)
{
    return launch_theta<T>(theta_args(c), u, v, out, mode, tau, c->st);
}

bool use_stream(wig2_ctx* c)
{
    if (c->theta_path == WIG2_THETA_GENERAL || !theta_stream_ok(theta_args(c))) return false;
    if (c->prm.precision == WIG2_BF16X2) return true;  // split-BF16 streaming kernel
    return c->theta_path == WIG2_THETA_STREAM || theta_stream_preferred(c->g.nk, c->elem);
}

// Single-operand Theta forms (streaming kernel or, for nk = 256 boxes, the
// panel kernel): 0 Theta x, 1 x + tau Theta x, 2 (y + x)/2 + tau/2 Theta x.
bool use_forms(wig2_ctx* c) { return use_stream(c) || theta_panel_ok(theta_args(c)); }

template <typename T>
hipError_t theta_form(wig2_ctx* c, const T* x, const T* y, T* out, int form, double tau)
{
    const ThetaArgs a = theta_args(c);
    if (theta_panel_ok(a)) return launch_theta_panel<T>(a, x, y, out, form, tau, c->st);
    return launch_theta_stream<T>(a, x, y, out, form, tau, c->st);
}

template <typename T>
hipError_t update_meanfield(wig2_ctx* c, const T* a, const T* b, double tau_b)
{
    hipError_t e = moments<T>(c, a, c->s0_d, nullptr, nullptr, nullptr);
    if (e != hipSuccess) return e;
    if (b) {
        e = moments<T>(c, b, c->s0b_d, nullptr, nullptr, nullptr);
        if (e != hipSuccess) return e;
    }
    return launch_meanfield(mf_args(c), c->s0_d, b ? c->s0b_d : nullptr, tau_b, c->sig1_d, c->sig2_d,
                            c->st);
}

// One step of the Lawson predictor-corrector (Sec. 4.1):
// a = A_tau f, b = A_tau Theta[f], f+ = a + (tau/2) Theta[a + tau b] + (tau/2) b.
template <typename T>
hipError_t step_lawson(wig2_ctx* c)
{
    T* f = static_cast<T*>(c->f);
    T* k1 = static_cast<T*>(c->k1);
    T* tmp = static_cast<T*>(c->tmp);
    const double tau = c->prm.dt;
    hipError_t e;
#define STEPCHK(x)                     \
    do {                               \
        e = (x);                       \
        if (e != hipSuccess) return e; \
    } while (0)
    auto ADV = [&](int dim, double sh, const T* in, T* out) {
        return timed(c, dim == 1 ? WIG2_PROF_ADVECT_X1 : WIG2_PROF_ADVECT_X2,
                     [&] { return advect<T>(c, dim, sh, in, out); });
    };
    auto TH = [&](const T* u, const T* v, T* out, int mode) {
        return timed(c, mode == 0 ? WIG2_PROF_THETA_STAGE1 : WIG2_PROF_THETA_STAGE2,
                     [&] { return theta<T>(c, u, v, out, mode, tau); });
    };
    auto MF = [&](const T* a, const T* b, double tb) {
        return timed(c, WIG2_PROF_MEANFIELD, [&] { return update_meanfield<T>(c, a, b, tb); });
    };
    auto THS = [&](const T* x, const T* y, T* out, int form) {
        return timed(c, form == 1 ? WIG2_PROF_THETA_STAGE1 : WIG2_PROF_THETA_STAGE2,
                     [&] { return theta_form<T>(c, x, y, out, form, tau); });
    };
    if (use_forms(c)) {
        // A_tau g = a + tau b for g = f + tau Theta f, so the corrector is
        // (y + x)/2 + (tau/2) Theta x with x = A_tau g and y = a = A_tau f
        if (c->meanfield) STEPCHK(MF(f, nullptr, 0.0));
        STEPCHK(THS(f, nullptr, k1, 1));
        STEPCHK(ADV(1, tau, f, tmp));
        STEPCHK(ADV(2, tau, tmp, f));
        STEPCHK(ADV(1, tau, k1, tmp));
        STEPCHK(ADV(2, tau, tmp, k1));
        if (c->meanfield) STEPCHK(MF(k1, nullptr, 0.0));
        STEPCHK(THS(k1, f, f, 2));
        return hipSuccess;
    }
    if (c->meanfield) STEPCHK(MF(f, nullptr, 0.0));
    STEPCHK(TH(f, nullptr, k1, 0));
    STEPCHK(ADV(1, tau, f, tmp));
    STEPCHK(ADV(2, tau, tmp, f));
    STEPCHK(ADV(1, tau, k1, tmp));
    STEPCHK(ADV(2, tau, tmp, k1));
    if (c->meanfield) STEPCHK(MF(f, k1, tau));
    STEPCHK(TH(f, k1, f, 1));
#undef STEPCHK
    return hipSuccess;
}


// Heun on Theta (V_eff frozen) from x into out (out may equal x); k1 is free.
template <typename T>
hipError_t heun_theta(wig2_ctx* c, T* x, T* out)
{
    T* k1 = static_cast<T*>(c->k1);
    const double tau = c->prm.dt;
    hipError_t e;
    if (c->meanfield) {
        e = timed(c, WIG2_PROF_MEANFIELD, [&] { return update_meanfield<T>(c, x, nullptr, 0.0); });
        if (e != hipSuccess) return e;
    }
    auto THS = [&](const T* a, const T* b, T* o, int form) {
        return timed(c, form == 3 ? WIG2_PROF_THETA_HEUN
                                  : form == 1 ? WIG2_PROF_THETA_STAGE1 : WIG2_PROF_THETA_STAGE2,
                     [&] { return theta_form<T>(c, a, b, o, form, tau); });
    };
    auto TH = [&](const T* u, const T* v, T* o, int mode) {
        return timed(c, mode == 0 ? WIG2_PROF_THETA_STAGE1 : WIG2_PROF_THETA_STAGE2,
                     [&] { return theta<T>(c, u, v, o, mode, tau); });
    };
    if (use_stream(c)) return THS(x, nullptr, out, 3);
    if (use_forms(c)) {
        if ((e = THS(x, nullptr, k1, 1)) != hipSuccess) return e;
        return THS(k1, x, out, 2);
    }
    if ((e = TH(x, nullptr, k1, 0)) != hipSuccess) return e;
    return TH(x, k1, out, 1);
}

// n >= 1 Strang steps A(tau/2) Heun A(tau/2) with A = (x2 sweep)(x1 sweep)
// on the way in and A = (x1 sweep)(x2 sweep) on the way out: the sweeps act
// on different axes with tensor-product operators, so the two orders are the
// same map (up to rounding).  The x1 half-sweep that ends a step and the one
// that begins the next are then consecutive and, where the line fits in
// registers, run as one two-pass launch (the same arithmetic without the
// intermediate HBM round trip): 3n + 1 state sweeps instead of 4n.  The state
// ends in c->f.
template <typename T>
hipError_t strang_steps(wig2_ctx* c, int64_t n)
{
    const double h = 0.5 * c->prm.dt;
    T* a = static_cast<T*>(c->f);
    T* b = static_cast<T*>(c->tmp);
    const double cpp = h / (c->g.mass * c->g.dx());
    const bool joint = c->fuse_sweeps && advect_in_registers(c->g.nx, c->g.periodic != 0, std::fabs(cpp) * c->pmax);
    auto sweep = [&](int dim, int passes, const T* in, T* out) {
        const int cls = passes == 2 ? WIG2_PROF_ADVECT_X1X1 : dim == 1 ? WIG2_PROF_ADVECT_X1 : WIG2_PROF_ADVECT_X2;
        return timed(c, cls, [&] {
            return launch_advect<T>(in, out, static_cast<T*>(c->work), c->g.nx, c->g.nk, dim, c->g.periodic != 0,
                                    cpp, std::fabs(cpp) * c->pmax, c->p_d, c->thomas_d, c->st, passes);
        });
    };
    // one sweep (or two along x1) from a into b, then b holds the state;
    // two x1 sweeps without the joint launch go through k1
    auto ADV = [&](int dim, int passes) {
        hipError_t e;
        if (passes == 2 && !joint) {
            T* k1 = static_cast<T*>(c->k1);
            if ((e = sweep(dim, 1, a, k1)) == hipSuccess) e = sweep(dim, 1, k1, b);
        } else {
            e = sweep(dim, passes, a, b);
        }
        std::swap(a, b);
        return e;
    };
    // 3n + 1 out-of-place sweeps; for even n the first Heun also writes the
    // other buffer so that the last sweep lands in c->f
    const bool flip = n % 2 == 0;
    hipError_t e;
    if ((e = ADV(1, 1)) != hipSuccess) return e;
    for (int64_t k = 0; k < n; ++k) {
        if ((e = ADV(2, 1)) != hipSuccess) return e;
        if (k == 0 && flip) {
            if ((e = heun_theta<T>(c, a, b)) != hipSuccess) return e;
            std::swap(a, b);
        } else if ((e = heun_theta<T>(c, a, a)) != hipSuccess) {
            return e;
        }
        if ((e = ADV(2, 1)) != hipSuccess) return e;
        if ((e = ADV(1, k + 1 < n ? 2 : 1)) != hipSuccess) return e;
    }
    return a == static_cast<T*>(c->f) ? hipSuccess : hipErrorUnknown;
}

template <typename T>
hipError_t run_steps(wig2_ctx* c, int64_t n)
{
    if (n <= 0) return hipSuccess;
    if (c->prm.scheme == WIG2_STRANG) return strang_steps<T>(c, n);
    hipError_t e = hipSuccess;
    for (int64_t k = 0; k < n && e == hipSuccess; ++k) e = step_lawson<T>(c);
    return e;
}

// ---- surrogate blocks -------------------------------------------------------

constexpr int kMaxParts = 1024;  // workgroups of the max-reduction

template <typename T>
hipError_t run_steps(wig2_ctx* c, int n, bool no_pair)
{
    c->no_pair = no_pair;
    hipError_t e = run_steps<T>(c, (int64_t)n);
    c->no_pair = false;
    return e;
}

// Mass and energy of a state (FP64 reductions, host sums as in wig2_observables).
template <typename T>
int scalar_obs(wig2_ctx* c, const T* f, double& mass, double& energy)
{
    const int nx = c->g.nx;
    const size_t np = (size_t)nx * nx;
    hipError_t e = moments<T>(c, f, c->s0_d, c->skin_d, nullptr, nullptr);
    if (e != hipSuccess) return fail(c, WIG2_EDEVICE, hipGetErrorString(e));
    std::vector<double> s0(np), sk(np);
    HIPCHK(c, hipMemcpyAsync(s0.data(), c->s0_d, np * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(sk.data(), c->skin_d, np * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    double m = 0.0, en = 0.0;
    for (int i1 = 0; i1 < nx; ++i1)
        for (int i2 = 0; i2 < nx; ++i2) {
            const size_t q = (size_t)i1 * nx + i2;
            const double vpot = (c->vext_x.empty() ? 0.0 : c->vext_x[i1] + c->vext_x[i2]) +
                                (c->v12pair.empty() ? 0.0 : c->v12pair[q]);
            m += s0[q];
            en += sk[q] + vpot * s0[q];
        }
    const double dx = c->g.dx();
    mass = dx * dx * m;
    energy = dx * dx * en;
    return WIG2_OK;
}

// max|a - b| and max|b| (d = a - b when d != NULL), synchronising.
template <typename T>
int diff_max(wig2_ctx* c, float* part, const T* a, const T* b, T* d, double& dmax, double& bmax)
{
    const long n = c->npts;
    const int nwg = (int)std::min<long>(kMaxParts, (n + 255) / 256);
    HIPCHK(c, launch_diff_max<T>(a, b, d, n, part, nwg, c->st));
    std::vector<float> h(2 * (size_t)nwg);
    HIPCHK(c, hipMemcpyAsync(h.data(), part, h.size() * sizeof(float), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    dmax = bmax = 0.0;
    for (int w = 0; w < nwg; ++w) {
        dmax = std::max(dmax, (double)h[2 * w]);
        bmax = std::max(bmax, (double)h[2 * w + 1]);
    }
    return WIG2_OK;
}

int ensure_sur_buffers(wig2_ctx* c)
{
    const size_t bytes = (size_t)c->npts * c->elem;
    if (!c->ft) HIPCHK(c, hipMalloc(&c->ft, bytes));
    if (!c->fs) HIPCHK(c, hipMalloc(&c->fs, bytes));
    return WIG2_OK;
}

long coprime_stride(long n)
{
    static const long primes[] = {1000003, 999983, 1000033, 999979};
    for (long q : primes)
        if (n % q != 0) return q % n == 0 ? 1 : q % n;
    return 1;
}

uint64_t splitmix(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// One pass over (ft, delta): minibatches of cfg.batch samples in a permuted
// order; train = Adam steps, else evaluation only.  Returns the mean loss.
template <typename T>
int sur_pass(wig2_surrogate* s, wig2_ctx* c, const T* ft, const T* delta, bool train, uint64_t salt,
             double& loss)
{
    const long n = c->npts;
    const long nwg_all = (n + 255) / 256 + (long)((n + s->cfg.batch - 1) / s->cfg.batch);
    if (nwg_all > s->lpart_cap) {
        if (s->lpart) hipFree(s->lpart);
        s->lpart = nullptr;
        HIPCHK(c, hipMalloc(&s->lpart, nwg_all * sizeof(float)));
        s->lpart_cap = nwg_all;
    }
    const long mul = coprime_stride(n);
    const long off = (long)(splitmix(s->cfg.seed ^ salt) % (uint64_t)n);
    long wg_used = 0;
    for (long k0 = 0; k0 < n; k0 += s->cfg.batch) {
        const long cnt = std::min<long>(s->cfg.batch, n - k0);
        const int nwg = (int)((cnt + 255) / 256);
        HIPCHK(c, launch_sur_batch<T>(ft, delta, c->g.nx, c->g.nk, n, k0, cnt, mul, off, s->sc, s->params,
                                      s->partial, s->lpart + wg_used, train, c->st));
        if (train) {
            ++s->updates;
            HIPCHK(c, launch_sur_adam(s->params, s->mom, s->var, s->pbf, s->partial, nwg, 2.0f / (float)cnt,
                                      (float)s->cfg.lr, (int)s->updates, nullptr, c->st));
        }
        wg_used += nwg;
    }
    std::vector<float> h((size_t)wg_used);
    HIPCHK(c, hipMemcpyAsync(h.data(), s->lpart, h.size() * sizeof(float), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    double sum = 0.0;
    for (float v : h) sum += v;
    loss = sum / (double)n;
    s->samples += n;
    return WIG2_OK;
}

template <typename T>
int sur_collect(wig2_surrogate* s, wig2_ctx* c, int blocks, bool train)
{
    T* f = static_cast<T*>(c->f);
    T* ft = static_cast<T*>(c->ft);
    T* fs = static_cast<T*>(c->fs);
    T* dl = static_cast<T*>(c->k1);  // Delta lives in k1 between steps
    const size_t bytes = (size_t)c->npts * sizeof(T);
    const int B = s->cfg.block;
    for (int b = 0; b < blocks; ++b) {
        HIPCHK(c, hipMemcpyAsync(ft, f, bytes, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(c, run_steps<T>(c, B, false));
        HIPCHK(c, hipMemcpyAsync(fs, f, bytes, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(c, hipMemcpyAsync(f, ft, bytes, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(c, run_steps<T>(c, B, true));
        double dmax, bmax, fmax, dummy;
        if (int r = diff_max<T>(c, s->maxpart, fs, f, dl, dmax, bmax)) return r;
        if (!s->scaled) {
            if (int r = diff_max<T>(c, s->maxpart, ft, ft, nullptr, dummy, fmax)) return r;
            s->sc.in_scale = fmax > 0.0 ? (float)(1.0 / fmax) : 1.f;
            s->sc.out_scale = dmax > 0.0 ? (float)dmax : 1.f;
            s->sc.inv_out_scale = 1.f / s->sc.out_scale;
            s->sc.u_feat = (float)(c->v12pair.empty() ? 0.0 : c->v12pair[0]);
            s->scaled = true;
        }
        double loss = 0.0;
        const int passes = train ? std::max(1, s->cfg.epochs) : 1;
        for (int ep = 0; ep < passes; ++ep) {
            const uint64_t salt = ((uint64_t)c->nstep << 20) ^ ((uint64_t)b << 8) ^ (uint64_t)ep;
            if (int r = sur_pass<T>(s, c, ft, dl, train, salt, loss)) return r;
        }
        if (train)
            s->train_loss = loss;
        else
            s->eval_loss = loss;
        HIPCHK(c, hipMemcpyAsync(f, fs, bytes, hipMemcpyDeviceToDevice, c->st));
        c->nstep += B;
        c->t += B * c->prm.dt;
    }
    return WIG2_OK;
}

// One block with the model attached (see wig2_surrogate_attach).
template <typename T>
int sur_block(wig2_ctx* c)
{
    const wig2_surrogate* s = c->sur;
    T* f = static_cast<T*>(c->f);
    T* ft = static_cast<T*>(c->ft);
    T* fs = static_cast<T*>(c->fs);
    const size_t bytes = (size_t)c->npts * sizeof(T);
    const int B = s->cfg.block;
    if (!c->sur_ref_ok) {
        if (int r = scalar_obs<T>(c, f, c->sur_mref, c->sur_eref)) return r;
        c->sur_ref_ok = true;
    }
    HIPCHK(c, hipMemcpyAsync(ft, f, bytes, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, run_steps<T>(c, B, true));
    HIPCHK(c, launch_sur_apply<T>(ft, f, c->g.nx, c->g.nk, s->sc, s->pbf, c->st));
    ++c->sur_blocks;
    ++c->sur_since;
    double m, en;
    if (int r = scalar_obs<T>(c, f, m, en)) return r;
    const double drift = std::max(std::fabs(m - c->sur_mref) / std::max(std::fabs(c->sur_mref), 1e-300),
                                  std::fabs(en - c->sur_eref) / std::max(std::fabs(c->sur_eref), 1e-300));
    const bool bad = !(drift <= c->sur_tol);
    const bool check = c->sur_every > 0 && c->sur_since >= c->sur_every;
    if (bad || check) {
        if (check) HIPCHK(c, hipMemcpyAsync(fs, f, bytes, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(c, hipMemcpyAsync(f, ft, bytes, hipMemcpyDeviceToDevice, c->st));
        HIPCHK(c, run_steps<T>(c, B, false));
        if (check) {
            double dmax, fmax;
            if (int r = diff_max<T>(c, s->maxpart, fs, f, nullptr, dmax, fmax)) return r;
            c->sur_last_err = fmax > 0.0 ? dmax / fmax : dmax;
            ++c->sur_checks;
            c->sur_since = 0;
        }
        if (bad) ++c->sur_fallbacks;
        if (int r = scalar_obs<T>(c, f, c->sur_mref, c->sur_eref)) return r;
    }
    c->nstep += B;
    c->t += B * c->prm.dt;
    return WIG2_OK;
}

int ensure_work(wig2_ctx* c)
{
    const double s = c->prm.scheme == WIG2_STRANG ? 0.5 * c->prm.dt : c->prm.dt;
    const double maxc = s * c->pmax / (c->g.mass * c->g.dx());
    if (c->work || advect_in_registers(c->g.nx, c->g.periodic != 0, maxc)) return 0;
    HIPCHK(c, hipMalloc(&c->work, (size_t)c->npts * c->elem));
    return 0;
}

}  // namespace

extern "C" {

const char* wig2_strerror(int code)
{
    switch (code) {
    case WIG2_OK: return "ok";
    case WIG2_EINVAL: return "invalid argument";
    case WIG2_ENOMEM: return "out of memory";
    case WIG2_EDEVICE: return "HIP device error";
    case WIG2_ESTATE: return "call out of order";
    case WIG2_ENOTSUP: return "not supported";
    case WIG2_ENUMERIC: return "non-finite value";
    default: return "unknown error";
    }
}

const char* wig2_last_error(const wig2_ctx* c) { return c ? c->err.c_str() : "null context"; }

int wig2_create(const wig2_grid* grid, const wig2_params* prm, void* hip_stream, wig2_ctx** out)
{
    if (!grid || !prm || !out) return WIG2_EINVAL;
    *out = nullptr;
    const wig2_grid& G = *grid;
    const wig2_params& P = *prm;
    if (G.nx < 4 || G.nk < 2 || !isfin(G.x_min) || !isfin(G.x_max) || !(G.x_max > G.x_min))
        return WIG2_EINVAL;
    if (!isfin(P.hbar) || !isfin(P.mass) || !isfin(P.dt) || !(P.hbar > 0) || !(P.mass > 0) ||
        !(P.dt > 0) || !isfin(P.meanfield_lambda))
        return WIG2_EINVAL;
    if (P.scheme != WIG2_STRANG && P.scheme != WIG2_LAWSON_PC) return WIG2_EINVAL;
    if (P.precision != WIG2_FP64 && P.precision != WIG2_FP32 && P.precision != WIG2_BF16X2)
        return WIG2_EINVAL;
    if (!G.periodic) {
        if (G.sem_cells < 1 || G.nk % G.sem_cells != 0 || !isfin(G.k_max) || !(G.k_max > 0))
            return WIG2_EINVAL;
    }
    if (P.xc && (!isfin(P.xc_n0) || !isfin(P.n_scale))) return WIG2_EINVAL;
    const bool panel = !G.periodic && G.nk == kPanelThetaNk;
    if (!theta_nk_ok(G.nk) && !panel) return WIG2_ENOTSUP;
    if (P.precision == WIG2_BF16X2 && G.nk % 32 != 0) return WIG2_ENOTSUP;
    if (!G.periodic && (P.meanfield_lambda != 0.0 || P.xc)) return WIG2_ENOTSUP;
    if (!G.periodic && !panel && P.precision == WIG2_BF16X2) return WIG2_ENOTSUP;

    wig2_ctx* c = new (std::nothrow) wig2_ctx();
    if (!c) return WIG2_ENOMEM;
    c->g = GridInfo{G.nx, G.nk, G.periodic ? 1 : 0, G.periodic ? 1 : G.sem_cells, G.x_min, G.x_max,
                    G.k_max, P.hbar, P.mass};
    c->prm = P;
    c->elem = P.precision == WIG2_FP64 ? 8 : 4;
    c->npts = (long)G.nx * G.nx * G.nk * G.nk;
    c->meanfield = P.meanfield_lambda != 0.0 || P.xc;
    auto bail = [&](int code) {
        wig2_destroy(c);
        return code;
    };
    if (hipGetDevice(&c->device) != hipSuccess) return bail(WIG2_EDEVICE);
    if (resolve_noalloc_scratch(c->device) != hipSuccess) return bail(WIG2_EDEVICE);
    if (hip_stream) {
        c->st = static_cast<hipStream_t>(hip_stream);
    } else {
        if (hipStreamCreateWithFlags(&c->st, hipStreamNonBlocking) != hipSuccess) return bail(WIG2_EDEVICE);
        c->own_stream = true;
    }
    const size_t bytes = (size_t)c->npts * c->elem;
    if (hipMalloc(&c->f_own, bytes) != hipSuccess || hipMalloc(&c->k1, bytes) != hipSuccess ||
        hipMalloc(&c->tmp, bytes) != hipSuccess)
        return bail(WIG2_ENOMEM);
    c->f = c->f_own;
    const int nx = G.nx, nk = G.nk;
    const size_t np = (size_t)nx * nx;
    if (dev_alloc(c, &c->p_d, nk) || dev_alloc(c, &c->w_d, nk) || dev_alloc(c, &c->thomas_d, nx) ||
        dev_alloc(c, &c->sig_ext_d, (size_t)nx * nk) || dev_alloc(c, &c->sig1_d, (size_t)nx * nk) ||
        dev_alloc(c, &c->sig2_d, (size_t)nx * nk) || dev_alloc(c, &c->kap_d, (size_t)nx * nk) ||
        dev_alloc(c, &c->v12pair_d, np) || dev_alloc(c, &c->sintab_d, (size_t)nk * nx) ||
        dev_alloc(c, &c->mf_dens_d, 2 * (size_t)nx) || dev_alloc(c, &c->mf_veff_d, 2 * (size_t)nx) ||
        dev_alloc(c, &c->s0_d, np) || dev_alloc(c, &c->s0b_d, np) || dev_alloc(c, &c->skin_d, np) ||
        dev_alloc(c, &c->s2_d, np) || dev_alloc(c, &c->rows_d, np * nk) ||
        dev_alloc(c, &c->f1_d, (size_t)nx * nk))
        return bail(WIG2_ENOMEM);
    if (!G.periodic && dev_alloc(c, &c->ksem_d, (size_t)nx * nk * nk)) return bail(WIG2_ENOMEM);
    if (panel && c->elem == 4 && dev_alloc(c, &c->ksem_f, (size_t)nx * nk * nk)) return bail(WIG2_ENOMEM);

    host_nodes(c->g, c->x, c->p, c->w);
    c->pmax = 0.0;
    for (double v : c->p) c->pmax = std::max(c->pmax, std::fabs(v));
    std::vector<double> th(nx, 0.0);
    {
        double m = 0.0;
        for (int i = 1; i < nx - 1; ++i) {
            m = 1.0 / (4.0 - m);
            th[i] = m;
        }
    }
    std::vector<double> sintab((size_t)nk * nx);
    for (int m = 0; m < nk; ++m)
        for (int d = 0; d < nx; ++d)
            sintab[(size_t)m * nx + d] = std::sin(2.0 * 3.141592653589793238462643383279502884 * m * d / nx);
    if (upload(c, c->p_d, c->p) || upload(c, c->w_d, c->w) || upload(c, c->thomas_d, th) ||
        upload(c, c->sintab_d, sintab))
        return bail(WIG2_EDEVICE);
    if (ensure_work(c)) return bail(WIG2_ENOMEM);
    *out = c;
    return WIG2_OK;
}

void wig2_destroy(wig2_ctx* c)
{
    if (!c) return;
    if (c->st) hipStreamSynchronize(c->st);
    void* bufs[] = {c->f_own, c->k1, c->tmp, c->work, c->p_d, c->w_d, c->thomas_d, c->sig_ext_d, c->sig1_d,
                    c->sig2_d, c->kap_d, c->ksem_d, c->ksem_f, c->v12pair_d, c->sintab_d,
                    c->mf_dens_d, c->mf_veff_d, c->s0_d, c->s0b_d, c->skin_d, c->s2_d, c->rows_d,
                    c->f1_d, c->ft, c->fs};
    for (void* b : bufs)
        if (b) hipFree(b);
    for (auto& pe : c->prof_ev) {
        hipEventDestroy(pe.second.first);
        hipEventDestroy(pe.second.second);
    }
    for (hipEvent_t e : c->ev_pool) hipEventDestroy(e);
    if (c->own_stream && c->st) hipStreamDestroy(c->st);
    delete c;
}

int wig2_set_potentials(wig2_ctx* c, wig2_fn1 v_ext, wig2_fn1 v12, void* user)
{
    if (!c) return WIG2_EINVAL;
    const GridInfo& g = c->g;
    const int nx = g.nx, nk = g.nk;
    const double L = g.L();
    auto V = [&](wig2_fn1 fn, double x) { return fn ? fn(x, user) : 0.0; };
    if (!g.periodic && v12) return fail(c, WIG2_ENOTSUP, "pair potential on a box needs the two-body SEM operator");
    c->vext_x.resize(nx);
    for (int i = 0; i < nx; ++i) c->vext_x[i] = V(v_ext, c->x[i]);
    c->v12pair.assign((size_t)nx * nx, 0.0);
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nx; ++j) {
            double r = c->x[i] - c->x[j];
            if (g.periodic) r -= L * std::floor((r + 0.5 * L) / L);
            c->v12pair[(size_t)i * nx + j] = V(v12, r);
        }
    for (double v : c->vext_x)
        if (!isfin(v)) return fail(c, WIG2_EINVAL, "V_ext returned a non-finite value");
    for (double v : c->v12pair)
        if (!isfin(v)) return fail(c, WIG2_EINVAL, "V12 returned a non-finite value");
    if (g.periodic) {
        std::vector<double> vy(2 * nk), vr(2 * nk), s, vh, kap;
        for (int j = 0; j < 2 * nk; ++j) {
            vy[j] = V(v_ext, g.x_min + L * j / (2 * nk));
            vr[j] = V(v12, -0.5 * L + L * j / (2 * nk));
            if (!isfin(vy[j]) || !isfin(vr[j])) return fail(c, WIG2_EINVAL, "non-finite potential sample");
        }
        host_symbol_ext(g, vy, s);
        host_pair_kernel(g, vr, vh, kap);
        double smax = 0.0;
        for (double v : s) smax = std::max(smax, std::fabs(v));
        c->band = 0;
        for (int m = 1; m < nk; ++m)
            for (int i = 0; i < nx; ++i)
                if (std::fabs(s[(size_t)i * nk + m]) > 1e-13 * smax) c->band = std::max(c->band, m);
        c->two_body = false;
        for (int m = 1; m < nk; ++m)
            if (vh[m] != 0.0) c->two_body = true;
        if (upload(c, c->sig_ext_d, s) || upload(c, c->kap_d, kap)) return WIG2_EDEVICE;
        if (c->meanfield) {
            if (upload(c, c->sig1_d, s) || upload(c, c->sig2_d, s)) return WIG2_EDEVICE;
        }
    } else {
        std::vector<double> K;
        host_sem_matrix(g, c->vext_x, K);
        if (upload(c, c->ksem_d, K)) return WIG2_EDEVICE;
        if (c->ksem_f) {
            const std::vector<float> Kf(K.begin(), K.end());
            HIPCHK(c, hipMemcpyAsync(c->ksem_f, Kf.data(), Kf.size() * sizeof(float), hipMemcpyHostToDevice, c->st));
            HIPCHK(c, hipStreamSynchronize(c->st));
        }
        c->two_body = false;
        c->band = nk;
    }
    if (upload(c, c->v12pair_d, c->v12pair)) return WIG2_EDEVICE;
    c->has_pot = true;
    c->err.clear();
    return WIG2_OK;
}

int wig2_set_state(wig2_ctx* c, const double* fh)
{
    if (!c || !fh) return WIG2_EINVAL;
    if (c->elem == 8) {
        HIPCHK(c, hipMemcpyAsync(c->f, fh, (size_t)c->npts * 8, hipMemcpyHostToDevice, c->st));
    } else {
        std::vector<float> tmp(c->npts);
        for (long i = 0; i < c->npts; ++i) tmp[i] = (float)fh[i];
        HIPCHK(c, hipMemcpyAsync(c->f, tmp.data(), (size_t)c->npts * 4, hipMemcpyHostToDevice, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    c->has_state = true;
    c->nstep = 0;
    c->t = 0.0;
    c->err.clear();
    return WIG2_OK;
}

int wig2_get_state(wig2_ctx* c, double* fh)
{
    if (!c || !fh) return WIG2_EINVAL;
    if (!c->has_state) return fail(c, WIG2_ESTATE, "no state");
    if (c->elem == 8) {
        HIPCHK(c, hipMemcpyAsync(fh, c->f, (size_t)c->npts * 8, hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
    } else {
        std::vector<float> tmp(c->npts);
        HIPCHK(c, hipMemcpyAsync(tmp.data(), c->f, (size_t)c->npts * 4, hipMemcpyDeviceToHost, c->st));
        HIPCHK(c, hipStreamSynchronize(c->st));
        for (long i = 0; i < c->npts; ++i) fh[i] = tmp[i];
    }
    return WIG2_OK;
}

int wig2_state_buffer(wig2_ctx* c, void** fd, int32_t* eb)
{
    if (!c || !fd) return WIG2_EINVAL;
    *fd = c->f;
    if (eb) *eb = c->elem;
    return WIG2_OK;
}

int wig2_bind_state(wig2_ctx* c, void* f_dev, int32_t dtype)
{
    if (!c) return WIG2_EINVAL;
    // work already queued on the context stream may still use the old buffer
    HIPCHK(c, hipStreamSynchronize(c->st));
    if (!f_dev) {
        c->f = c->f_own;
        c->has_state = false;
        c->err.clear();
        return WIG2_OK;
    }
    const int32_t want = c->elem == 8 ? WIG2_FP64 : WIG2_FP32;
    if (dtype != want)
        return fail(c, WIG2_EINVAL, c->elem == 8 ? "bind_state: this context steps an FP64 state (dtype WIG2_FP64)"
                                                 : "bind_state: this context steps an FP32 state (dtype WIG2_FP32)");
    if (reinterpret_cast<uintptr_t>(f_dev) % 16 != 0)
        return fail(c, WIG2_EINVAL, "bind_state: the buffer must be 16-byte aligned");
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, f_dev) != hipSuccess || attr.type != hipMemoryTypeDevice ||
        attr.device != c->device) {
        (void)hipGetLastError();
        return fail(c, WIG2_EINVAL, "bind_state: not device memory of this context's device");
    }
    c->f = f_dev;
    c->has_state = true;
    c->nstep = 0;
    c->t = 0.0;
    c->err.clear();
    return WIG2_OK;
}

int wig2_state_written(wig2_ctx* c)
{
    if (!c) return WIG2_EINVAL;
    c->has_state = true;
    c->nstep = 0;
    c->t = 0.0;
    return WIG2_OK;
}

int wig2_step(wig2_ctx* c, int64_t n)
{
    if (!c || n < 0) return WIG2_EINVAL;
    if (!c->has_state || !c->has_pot) return fail(c, WIG2_ESTATE, "set the state and the potentials first");
    if (c->sur) {
        const int B = c->sur->cfg.block;
        for (; n >= B; n -= B)
            if (int r = c->elem == 8 ? sur_block<double>(c) : sur_block<float>(c)) return r;
    }
    if (n == 0) return WIG2_OK;
    hipError_t e = c->elem == 8 ? run_steps<double>(c, n) : run_steps<float>(c, n);
    if (e != hipSuccess) return fail(c, e == hipErrorNotSupported ? WIG2_ENOTSUP : WIG2_EDEVICE,
                                     std::string("step: ") + hipGetErrorString(e));
    c->nstep += n;
    c->t += (double)n * c->prm.dt;
    return WIG2_OK;
}

int wig2_theta(wig2_ctx* c, const void* in, void* out)
{
    if (!c || !in || !out) return WIG2_EINVAL;
    if (!c->has_pot) return fail(c, WIG2_ESTATE, "set the potentials first");
    if (in == out && theta_panel_ok(theta_args(c)) && (c->elem == 8 || c->prm.precision == WIG2_BF16X2))
        return fail(c, WIG2_EINVAL, "theta: in and out must differ for nk = 256 boxes in FP64 / BF16X2");
    hipError_t e;
    if (c->elem == 8) {
        if (c->meanfield && (e = update_meanfield<double>(c, (const double*)in, nullptr, 0.0)) != hipSuccess)
            return fail(c, WIG2_EDEVICE, hipGetErrorString(e));
        e = use_forms(c) ? theta_form<double>(c, (const double*)in, nullptr, (double*)out, 0, c->prm.dt)
                         : theta<double>(c, (const double*)in, nullptr, (double*)out, 0, c->prm.dt);
    } else {
        if (c->meanfield && (e = update_meanfield<float>(c, (const float*)in, nullptr, 0.0)) != hipSuccess)
            return fail(c, WIG2_EDEVICE, hipGetErrorString(e));
        e = use_forms(c) ? theta_form<float>(c, (const float*)in, nullptr, (float*)out, 0, c->prm.dt)
                         : theta<float>(c, (const float*)in, nullptr, (float*)out, 0, c->prm.dt);
    }
    if (e != hipSuccess) return fail(c, e == hipErrorNotSupported ? WIG2_ENOTSUP : WIG2_EDEVICE,
                                     std::string("theta: ") + hipGetErrorString(e));
    return WIG2_OK;
}

int wig2_advect(wig2_ctx* c, int32_t dim, double s, const void* in, void* out)
{
    if (!c || !in || !out || in == out || (dim != 1 && dim != 2) || !isfin(s)) return WIG2_EINVAL;
    const double maxc = std::fabs(s) * c->pmax / (c->g.mass * c->g.dx());
    if (!advect_in_registers(c->g.nx, c->g.periodic != 0, maxc) && !c->work)
        HIPCHK(c, hipMalloc(&c->work, (size_t)c->npts * c->elem));
    hipError_t e = c->elem == 8 ? advect<double>(c, dim, s, (const double*)in, (double*)out)
                                : advect<float>(c, dim, s, (const float*)in, (float*)out);
    if (e != hipSuccess) return fail(c, WIG2_EDEVICE, std::string("advect: ") + hipGetErrorString(e));
    return WIG2_OK;
}

int wig2_advect_noalloc(wig2_ctx* c, int32_t dim, double s, const void* in, void* out)
{
    if (!c || !in || !out || in == out || (dim != 1 && dim != 2) || !isfin(s)) return WIG2_EINVAL;
    const double cpp = s / (c->g.mass * c->g.dx());
    const double maxc = std::fabs(cpp) * c->pmax;
    void* ws = nullptr;
    if (!advect_in_registers(c->g.nx, c->g.periodic != 0, maxc)) {
        // the general sweep writes every coefficient of a line before it reads
        // one, so the scratch needs no clearing between calls
        if ((size_t)c->npts * c->elem > kNoAllocScratchBytes)
            return fail(c, WIG2_EINVAL, "advect_noalloc: this sweep needs a coefficient buffer of the "
                                        "state's size, larger than the 64 MiB static scratch");
        ws = noalloc_scratch(c->device);
        if (!ws) return fail(c, WIG2_ESTATE, "advect_noalloc: scratch address not resolved on this device");
    }
    hipError_t e = c->elem == 8
                       ? launch_advect<double>((const double*)in, (double*)out, (double*)ws, c->g.nx, c->g.nk,
                                               dim, c->g.periodic != 0, cpp, maxc, c->p_d, c->thomas_d, c->st)
                       : launch_advect<float>((const float*)in, (float*)out, (float*)ws, c->g.nx, c->g.nk,
                                              dim, c->g.periodic != 0, cpp, maxc, c->p_d, c->thomas_d, c->st);
    if (e != hipSuccess) return fail(c, WIG2_EDEVICE, "advect_noalloc: launch failed");
    return WIG2_OK;
}

int wig2_set_sweep_fusion(wig2_ctx* c, int32_t enable)
{
    if (!c) return WIG2_EINVAL;
    c->fuse_sweeps = enable != 0;
    return WIG2_OK;
}

int wig2_set_theta_path(wig2_ctx* c, int32_t path)
{
    if (!c || path < WIG2_THETA_AUTO || path > WIG2_THETA_STREAM) return WIG2_EINVAL;
    if (path == WIG2_THETA_STREAM && c->has_pot && !theta_stream_ok(theta_args(c)))
        return fail(c, WIG2_ENOTSUP, "streaming Theta needs a torus, nk in {32,48,64,96,128} (BF16X2: "
                                     "{32,64,96,128}) and a single-body band of at most 4 modes");
    c->theta_path = path;
    return WIG2_OK;
}

int wig2_theta_path(const wig2_ctx* c)
{
    if (!c) return WIG2_EINVAL;
    if (!c->has_pot) return WIG2_ESTATE;
    wig2_ctx* m = const_cast<wig2_ctx*>(c);
    if (theta_panel_ok(theta_args(m))) return WIG2_THETA_PANEL;
    return use_stream(m) ? WIG2_THETA_STREAM : WIG2_THETA_GENERAL;
}

int wig2_nodes(const wig2_ctx* c, double* x, double* p, double* w)
{
    if (!c) return WIG2_EINVAL;
    if (x) std::copy(c->x.begin(), c->x.end(), x);
    if (p) std::copy(c->p.begin(), c->p.end(), p);
    if (w) std::copy(c->w.begin(), c->w.end(), w);
    return WIG2_OK;
}

int wig2_profile(wig2_ctx* c, int32_t enable)
{
    if (!c) return WIG2_EINVAL;
    c->prof = enable != 0;
    return WIG2_OK;
}

int wig2_profile_read(wig2_ctx* c, double* ms, int64_t* counts, int32_t reset)
{
    if (!c) return WIG2_EINVAL;
    HIPCHK(c, hipStreamSynchronize(c->st));
    for (auto& pe : c->prof_ev) {
        float v = 0.f;
        if (hipEventElapsedTime(&v, pe.second.first, pe.second.second) == hipSuccess) {
            c->prof_ms[pe.first] += v;
            c->prof_cnt[pe.first] += 1;
        }
        c->ev_pool.push_back(pe.second.first);
        c->ev_pool.push_back(pe.second.second);
    }
    c->prof_ev.clear();
    for (int k = 0; k < WIG2_PROF_N; ++k) {
        if (ms) ms[k] = c->prof_ms[k];
        if (counts) counts[k] = c->prof_cnt[k];
        if (reset) {
            c->prof_ms[k] = 0.0;
            c->prof_cnt[k] = 0;
        }
    }
    return WIG2_OK;
}

int wig2_band(const wig2_ctx* c)
{
    if (!c) return WIG2_EINVAL;
    return c->meanfield ? c->g.nk - 1 : std::min(c->band, c->g.nk - 1);
}

int wig2_observables(wig2_ctx* c, wig2_obs* o, double* n1, double* n12, double* f1)
{
    if (!c || !o) return WIG2_EINVAL;
    if (!c->has_state) return fail(c, WIG2_ESTATE, "no state");
    const int nx = c->g.nx, nk = c->g.nk;
    const size_t np = (size_t)nx * nx;
    hipError_t e = c->elem == 8
                       ? moments<double>(c, (const double*)c->f, c->s0_d, c->skin_d, c->s2_d, c->rows_d)
                       : moments<float>(c, (const float*)c->f, c->s0_d, c->skin_d, c->s2_d, c->rows_d);
    if (e != hipSuccess) return fail(c, WIG2_EDEVICE, hipGetErrorString(e));
    const double dx = c->g.dx();
    HIPCHK(c, launch_reduce_rows(c->rows_d, nx, nk, dx, c->f1_d, c->st));
    std::vector<double> s0(np), sk(np), s2(np), hf1((size_t)nx * nk);
    HIPCHK(c, hipMemcpyAsync(s0.data(), c->s0_d, np * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(sk.data(), c->skin_d, np * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(s2.data(), c->s2_d, np * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipMemcpyAsync(hf1.data(), c->f1_d, hf1.size() * 8, hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    double mass = 0.0, en = 0.0, l2 = 0.0;
    for (int i1 = 0; i1 < nx; ++i1)
        for (int i2 = 0; i2 < nx; ++i2) {
            const size_t q = (size_t)i1 * nx + i2;
            const double vpot = (c->vext_x.empty() ? 0.0 : c->vext_x[i1] + c->vext_x[i2]) +
                                (c->v12pair.empty() ? 0.0 : c->v12pair[q]);
            mass += s0[q];
            en += sk[q] + vpot * s0[q];
            l2 += s2[q];
        }
    o->step = c->nstep;
    o->t = c->t;
    o->mass = dx * dx * mass;
    o->energy = dx * dx * en;
    o->l2 = dx * dx * l2;
    std::vector<double> occ;
    o->entropy_vn = host_entropy(c->g, hf1, occ);
    o->fallbacks = (int32_t)c->sur_fallbacks;
    if (n12) std::copy(s0.begin(), s0.end(), n12);
    if (n1)
        for (int i1 = 0; i1 < nx; ++i1) {
            double s = 0.0;
            for (int i2 = 0; i2 < nx; ++i2) s += s0[(size_t)i1 * nx + i2];
            n1[i1] = dx * s;
        }
    if (f1) std::copy(hf1.begin(), hf1.end(), f1);
    if (!isfin(o->mass) || !isfin(o->energy) || !isfin(o->l2))
        return fail(c, WIG2_ENUMERIC, "non-finite observable");
    return WIG2_OK;
}

// ---- learned surrogate ---------------------------------------------------------

namespace {
int sfail(wig2_surrogate* s, int code, const std::string& m)
{
    if (s) s->err = m;
    return code;
}
unsigned short host_bf16(float v)
{
    unsigned u;
    std::memcpy(&u, &v, 4);
    return (unsigned short)((u + 0x7FFFu + ((u >> 16) & 1u)) >> 16);
}
int sur_ctx_ok(wig2_surrogate* s, wig2_ctx* c)
{
    if (!c->has_state || !c->has_pot) return sfail(s, WIG2_ESTATE, "context needs state and potentials");
    if (!c->g.periodic || !c->two_body || c->meanfield)
        return sfail(s, WIG2_ENOTSUP, "surrogate needs a torus context with a pair potential, no mean field");
    if (c->prm.precision == WIG2_BF16X2) return sfail(s, WIG2_ENOTSUP, "surrogate needs FP64 or FP32 state");
    if (s->dt != 0.0 && std::fabs(s->dt - c->prm.dt) > 1e-15 * s->dt)
        return sfail(s, WIG2_EINVAL, "model was trained with another dt");
    return WIG2_OK;
}
}  // namespace

const char* wig2_surrogate_last_error(const wig2_surrogate* s) { return s ? s->err.c_str() : "null model"; }

int wig2_surrogate_create(const wig2_train_cfg* cfg, wig2_surrogate** out)
{
    if (!cfg || !out) return WIG2_EINVAL;
    *out = nullptr;
    if (cfg->radius != kSurR || cfg->hidden != kSurH) return WIG2_ENOTSUP;
    if (cfg->block < 1 || cfg->epochs < 0 || cfg->batch < 256 || cfg->batch % 256 || !(cfg->lr > 0.0))
        return WIG2_EINVAL;
    wig2_surrogate* s = new (std::nothrow) wig2_surrogate();
    if (!s) return WIG2_ENOMEM;
    s->cfg = *cfg;
    hipGetDevice(&s->device);
    const int nwg = cfg->batch / 256;
    bool ok = hipMalloc((void**)&s->params, kSurP * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->mom, kSurP * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->var, kSurP * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->pbf, kSurP * sizeof(unsigned short)) == hipSuccess &&
              hipMalloc((void**)&s->grad, kSurP * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->maxpart, 2 * kMaxParts * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->partial, (size_t)nwg * kSurP * sizeof(float)) == hipSuccess;
    if (!ok) {
        wig2_surrogate_destroy(s);
        return WIG2_ENOMEM;
    }
    // Xavier-uniform weights, zero biases and linear path
    std::vector<float> p(kSurP, 0.f);
    const int D = kSurD, H = kSurH;
    auto fill = [&](int off, int n, int fan_in, int fan_out) {
        const double a = std::sqrt(6.0 / (fan_in + fan_out));
        for (int j = 0; j < n; ++j) {
            const double u = (double)(splitmix(cfg->seed * 0x100000001B3ull + (uint64_t)(off + j)) >> 11) *
                             (1.0 / 9007199254740992.0);
            p[(size_t)off + j] = (float)((2.0 * u - 1.0) * a);
        }
    };
    fill(0, H * D, D, H);                              // W1
    fill(H * D + H, H * H, H, H);                      // W2
    fill(H * D + H + H * H + H, H, H, 1);              // w3
    if (int r = wig2_surrogate_set_params(s, p.data(), nullptr)) {
        wig2_surrogate_destroy(s);
        return r;
    }
    *out = s;
    return WIG2_OK;
}

void wig2_surrogate_destroy(wig2_surrogate* s)
{
    if (!s) return;
    void* bufs[] = {s->params, s->mom, s->var, s->pbf, s->partial, s->lpart, s->grad, s->maxpart};
    for (void* b : bufs)
        if (b) hipFree(b);
    delete s;
}

int wig2_surrogate_get_params(const wig2_surrogate* s, float* params, float* scales)
{
    if (!s) return WIG2_EINVAL;
    if (params && hipMemcpy(params, s->params, kSurP * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return WIG2_EDEVICE;
    if (scales) {
        scales[0] = s->sc.in_scale;
        scales[1] = s->sc.out_scale;
        scales[2] = s->sc.u_feat;
    }
    return WIG2_OK;
}

int wig2_surrogate_set_params(wig2_surrogate* s, const float* params, const float* scales)
{
    if (!s) return WIG2_EINVAL;
    if (params) {
        std::vector<unsigned short> b(kSurP);
        for (int j = 0; j < kSurP; ++j) {
            if (!std::isfinite(params[j])) return sfail(s, WIG2_EINVAL, "non-finite parameter");
            b[j] = host_bf16(params[j]);
        }
        const std::vector<float> z(kSurP, 0.f);
        if (hipMemcpy(s->params, params, kSurP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(s->pbf, b.data(), kSurP * sizeof(unsigned short), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(s->mom, z.data(), kSurP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(s->var, z.data(), kSurP * sizeof(float), hipMemcpyHostToDevice) != hipSuccess)
            return sfail(s, WIG2_EDEVICE, "parameter upload failed");
        s->updates = 0;
    }
    if (scales) {
        if (!(scales[0] > 0.f) || !(scales[1] > 0.f) || !std::isfinite(scales[2]))
            return sfail(s, WIG2_EINVAL, "scales must be positive (in, out) and finite (U)");
        s->sc.in_scale = scales[0];
        s->sc.out_scale = scales[1];
        s->sc.inv_out_scale = 1.f / scales[1];
        s->sc.u_feat = scales[2];
        s->scaled = true;
    }
    return WIG2_OK;
}

int wig2_surrogate_stats(const wig2_surrogate* s, double* train_loss, double* eval_loss, int64_t* updates,
                         int64_t* samples)
{
    if (!s) return WIG2_EINVAL;
    if (train_loss) *train_loss = s->train_loss;
    if (eval_loss) *eval_loss = s->eval_loss;
    if (updates) *updates = s->updates;
    if (samples) *samples = s->samples;
    return WIG2_OK;
}

int wig2_surrogate_collect(wig2_surrogate* s, wig2_ctx* c, int32_t blocks, int32_t train)
{
    if (!s || !c || blocks < 0) return WIG2_EINVAL;
    if (int r = sur_ctx_ok(s, c)) return r;
    if (c->sur) return sfail(s, WIG2_ESTATE, "detach the model from the context first");
    if (int r = ensure_sur_buffers(c)) return sfail(s, r, c->err);
    if (s->dt == 0.0) s->dt = c->prm.dt;
    const int r = c->elem == 8 ? sur_collect<double>(s, c, blocks, train != 0)
                               : sur_collect<float>(s, c, blocks, train != 0);
    return r ? sfail(s, r, c->err) : WIG2_OK;
}

int wig2_surrogate_grad(wig2_surrogate* s, wig2_ctx* c, const void* ft, const void* delta, float* grad,
                        double* loss)
{
    if (!s || !c || !ft || !delta || !grad) return WIG2_EINVAL;
    const long n = c->npts;
    if (n > (1l << 22)) return sfail(s, WIG2_EINVAL, "gradient check limited to 2^22 points");
    const int nwg = (int)((n + 255) / 256);
    float* part = nullptr;
    float* lp = nullptr;
    if (hipMalloc((void**)&part, (size_t)nwg * kSurP * sizeof(float)) != hipSuccess ||
        hipMalloc((void**)&lp, (size_t)nwg * sizeof(float)) != hipSuccess) {
        if (part) hipFree(part);
        return WIG2_ENOMEM;
    }
    hipError_t e = c->elem == 8
                       ? launch_sur_batch<double>((const double*)ft, (const double*)delta, c->g.nx, c->g.nk, n, 0,
                                                  n, 1, 0, s->sc, s->params, part, lp, true, c->st)
                       : launch_sur_batch<float>((const float*)ft, (const float*)delta, c->g.nx, c->g.nk, n, 0, n,
                                                 1, 0, s->sc, s->params, part, lp, true, c->st);
    if (e == hipSuccess)
        e = launch_sur_adam(s->params, s->mom, s->var, s->pbf, part, nwg, 2.0f / (float)n, 0.f, 1, s->grad,
                            c->st);
    std::vector<float> hl((size_t)nwg);
    if (e == hipSuccess) e = hipMemcpyAsync(grad, s->grad, kSurP * sizeof(float), hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipMemcpyAsync(hl.data(), lp, hl.size() * sizeof(float), hipMemcpyDeviceToHost, c->st);
    if (e == hipSuccess) e = hipStreamSynchronize(c->st);
    hipFree(part);
    hipFree(lp);
    if (e != hipSuccess) return sfail(s, WIG2_EDEVICE, hipGetErrorString(e));
    if (loss) {
        double sum = 0.0;
        for (float v : hl) sum += v;
        *loss = sum / (double)n;
    }
    return WIG2_OK;
}

int wig2_surrogate_attach(wig2_ctx* c, const wig2_surrogate* s, double drift_tol, int32_t every)
{
    if (!c || !s || !(drift_tol >= 0.0) || every < 0) return WIG2_EINVAL;
    wig2_surrogate* ms = const_cast<wig2_surrogate*>(s);
    if (int r = sur_ctx_ok(ms, c)) return fail(c, r, s->err);
    if (!s->scaled) return fail(c, WIG2_ESTATE, "the model has no scales yet (collect or set them first)");
    if (int r = ensure_sur_buffers(c)) return r;
    c->sur = s;
    c->sur_tol = drift_tol;
    c->sur_every = every;
    c->sur_since = 0;
    c->sur_blocks = c->sur_fallbacks = c->sur_checks = 0;
    c->sur_last_err = -1.0;
    c->sur_ref_ok = false;
    return WIG2_OK;
}

int wig2_surrogate_detach(wig2_ctx* c)
{
    if (!c) return WIG2_EINVAL;
    c->sur = nullptr;
    return WIG2_OK;
}

int wig2_surrogate_report(const wig2_ctx* c, int64_t* blocks, int64_t* fallbacks, int64_t* checks,
                          double* last_check_eps)
{
    if (!c) return WIG2_EINVAL;
    if (blocks) *blocks = c->sur_blocks;
    if (fallbacks) *fallbacks = c->sur_fallbacks;
    if (checks) *checks = c->sur_checks;
    if (last_check_eps) *last_check_eps = c->sur_last_err;
    return WIG2_OK;
}

}  // extern "C"
