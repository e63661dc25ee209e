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
    double* fft_sym_d = nullptr;  // FFT Theta path: plane symbols, 3 nx (2 nk)
    double *ksem_d = nullptr, *v12pair_d = nullptr, *sintab_d = nullptr;
    int hartree = WIG2_HARTREE_PAIR;
    double* hart_d = nullptr;  // [nx][nx] Hartree kernel of the mean field
    float* ksem_f = nullptr;  // FP32 copy of the SEM matrices (nk = 256, FP32 / BF16X2)
    // box with a mean field: the SEM matrices of V_ext + V_eff,j per particle,
    // rebuilt from the factor tables on every update
    double *kmf1_d = nullptr, *kmf2_d = nullptr, *semE_d = nullptr, *semQ_d = nullptr;
    float *kmf1_f = nullptr, *kmf2_f = nullptr;
    double sem_pref = 0.0;
    // box with a pair potential: the two-body SEM operator's tables (element
    // type of the state), its per-chunk workspaces and a state-sized
    // accumulator for calls whose output aliases an input
    bool sem12 = false;
    void *s12_wa = nullptr, *s12_wb = nullptr, *s12_wc = nullptr, *s12_wd = nullptr, *s12_dt = nullptr;
    void *s12_wr = nullptr, *s12_wh = nullptr, *s12_acc = nullptr;
    long s12_chunk = 0;
    int ncu = 256;
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
    unsigned short* sur_buf = nullptr;  // inference activations: features and two layer buffers
    const wig2_surrogate* sur = nullptr;
    double sur_tol = 0.0;
    int sur_every = 0, sur_since = 0;
    int64_t sur_blocks = 0, sur_fallbacks = 0, sur_checks = 0;
    double sur_last_err = -1.0;
    bool sur_ref_ok = false;
    double sur_mref = 0.0, sur_eref = 0.0;
};

// One layer of the surrogate: a convolution along `axis` (0: p1, 1: p2,
// 2: x1, 3: x2) with K taps; W at params[woff] ([16][K][16]), its bias at
// params[woff + 256 K]; packed A fragments at frag[foff].
struct SurLayer {
    int axis, K;
    long woff, foff;
};

struct wig2_surrogate {
    int device = 0;
    wig2_train_cfg cfg{};
    std::vector<SurLayer> layers;
    long P = 0, head_off = 0, frag_total = 0;
    float* params = nullptr;  // FP32 master weights (layers, then the head w_o[16], b_o, a[16])
    float* mom = nullptr;
    float* var = nullptr;
    float* grad = nullptr;
    unsigned short* frag_f = nullptr;  // bf16 A fragments, forward
    unsigned short* frag_b = nullptr;  // bf16 A fragments, input gradient (transposed, flipped)
    float* part = nullptr;             // per-workgroup gradient sums
    size_t part_cap = 0;
    float* lpart = nullptr;            // per-workgroup loss sums
    size_t lpart_cap = 0;
    float* maxpart = nullptr;          // [2 * kMaxParts]
    long act_cap = 0;                  // training activations, points
    std::vector<unsigned short*> h;    // h[0] = features .. h[L]
    std::vector<unsigned short*> t;    // tanh outputs of the layers
    float* dh[2] = {nullptr, nullptr};
    int grid = 1024;
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
    a.v12pair = c->hart_d;
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
    a.fft_sym = c->fft_sym_d;
    a.ksem_t = nullptr;
    if (!c->g.periodic && c->g.nk == kPanelThetaNk)
        a.ksem_t = c->elem == 8 ? (const void*)c->ksem_d : (const void*)c->ksem_f;
    if (!c->g.periodic && c->meanfield) {
        a.ksem = c->kmf1_d;
        a.ksem2 = c->kmf2_d;
        if (c->g.nk == kPanelThetaNk) {
            a.ksem_t = c->elem == 8 ? (const void*)c->kmf1_d : (const void*)c->kmf1_f;
            a.ksem2_t = c->elem == 8 ? (const void*)c->kmf2_d : (const void*)c->kmf2_f;
        }
    }
    return a;
}

// Box with a pair potential: the two-body SEM operator (Sec. 3.2.2) is added
// to the single-body kernel's result.  `single` writes out = base + alpha
// Theta_1,2 x with x = u + beta v; this adds alpha Theta_12 x.  When out is
// neither u nor v the single-body kernel runs first and the last product of
// every chunk of planes accumulates onto out; otherwise Theta_12 x is formed
// first (into the accumulator) so that the inputs are read before out is
// written.
Sem12Args sem12_args(const wig2_ctx* c)
{
    return Sem12Args{c->g.nx, c->g.nk, c->ncu, c->s12_wa, c->s12_wb, c->s12_wc, c->s12_wd, c->s12_dt};
}

template <typename T, typename F>
hipError_t with_pair_sem(wig2_ctx* c, const T* u, const T* v, double beta, double alpha, T* out, F&& single)
{
    if (!c->sem12 || c->no_pair) return single();
    const long np = (long)c->g.nx * c->g.nx;
    const Sem12Args a = sem12_args(c);
    T* wr = static_cast<T*>(c->s12_wr);
    T* wh = static_cast<T*>(c->s12_wh);
    const bool direct = out != u && out != v;
    T* dst = direct ? out : static_cast<T*>(c->s12_acc);
    hipError_t e;
    if (direct && (e = single()) != hipSuccess) return e;
    e = timed(c, WIG2_PROF_PAIR_SEM, [&] {
        for (long p0 = 0; p0 < np; p0 += c->s12_chunk) {
            const long n = std::min(c->s12_chunk, np - p0);
            hipError_t e2 = launch_sem12_pre<T>(a, u, v, beta, p0, n, wr, wh, c->st);
            if (e2 == hipSuccess) e2 = launch_sem12_post<T>(a, wr, dst, alpha, direct, p0, n, c->st);
            if (e2 != hipSuccess) return e2;
        }
        return hipSuccess;
    });
    if (e != hipSuccess) return e;
    if (direct) return hipSuccess;
    if ((e = single()) != hipSuccess) return e;
    return launch_sem12_add<T>(dst, out, c->npts, c->ncu, c->st);
}

bool use_fft(const wig2_ctx* c) { return c->theta_path == WIG2_THETA_FFT; }

// mode 0: out = Theta u; mode 1: out = u + tau/2 (v + Theta (u + tau v))
template <typename T>
hipError_t theta(wig2_ctx* c, const T* u, const T* v, T* out, int mode, double tau)
{
    if (use_fft(c)) return launch_theta_fft<T>(theta_args(c), u, v, out, mode, tau, c->st);
    return with_pair_sem<T>(c, u, mode == 1 ? v : nullptr, mode == 1 ? tau : 0.0, mode == 1 ? 0.5 * tau : 1.0, out,
                            [&] { return launch_theta<T>(theta_args(c), u, v, out, mode, tau, c->st); });
}

bool use_stream(wig2_ctx* c)
{
    if (c->theta_path == WIG2_THETA_GENERAL || use_fft(c) || !theta_stream_ok(theta_args(c))) return false;
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
    if (theta_panel_ok(a)) {
        const double alpha = form == 0 ? 1.0 : form == 1 ? tau : 0.5 * tau;
        return with_pair_sem<T>(c, x, nullptr, 0.0, alpha, out,
                                [&] { return launch_theta_panel<T>(a, x, y, out, form, tau, c->st); });
    }
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
    if (c->g.periodic)
        return launch_meanfield(mf_args(c), c->s0_d, b ? c->s0b_d : nullptr, tau_b, c->sig1_d, c->sig2_d, c->st);
    // box: V_eff,j, then the SEM matrices of V_ext + V_eff,j
    e = launch_meanfield_potential(mf_args(c), c->s0_d, b ? c->s0b_d : nullptr, tau_b, c->st);
    if (e != hipSuccess) return e;
    const int nodes = c->g.nk / c->g.cells;
    const SemMfArgs sa{c->g.nx, c->g.nk, nodes, c->sem_pref, c->ksem_d, c->mf_veff_d,
                       c->semE_d, c->semQ_d, c->kmf1_d, c->kmf2_d};
    return launch_meanfield_sem(sa, c->kmf1_f, c->kmf2_f, c->st);
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
    // general kernel: the whole Heun step in one pass where it has that form
    // (torus), else its two stages (also the FFT path's form)
    if (!use_fft(c) && theta_heun_general_ok(theta_args(c)))
        return timed(c, WIG2_PROF_THETA_HEUN,
                     [&] { return launch_theta_heun<T>(theta_args(c), x, out, tau, c->st); });
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

int ensure_sur_buffers(wig2_ctx* c, bool inference = false)
{
    const size_t bytes = (size_t)c->npts * c->elem;
    if (!c->ft) HIPCHK(c, hipMalloc(&c->ft, bytes));
    if (!c->fs) HIPCHK(c, hipMalloc(&c->fs, bytes));
    if (inference && !c->sur_buf)
        HIPCHK(c, hipMalloc((void**)&c->sur_buf, 3 * (size_t)c->npts * kSurC * sizeof(unsigned short)));
    return WIG2_OK;
}

uint64_t splitmix(uint64_t x)
{
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// Axis geometry of a surrogate convolution on an nx^2 x nk^2 grid.
SurAxis sur_axis(int axis, int nx, int nk)
{
    const long nk2 = (long)nk * nk;
    SurAxis g{};
    if (axis == 1) {  // p2 = n2, tiles run along n1
        g.Sa = 1; g.La = nk; g.periodic = 0; g.Sl = nk; g.Ll = nk;
        g.R = (long)nx * nx; g.rdiv = nx; g.rs_hi = nx * nk2; g.rs_lo = nk2;
    } else if (axis == 0) {  // p1 = n1, tiles run along n2
        g.Sa = nk; g.La = nk; g.periodic = 0; g.Sl = 1; g.Ll = nk;
        g.R = (long)nx * nx; g.rdiv = nx; g.rs_hi = nx * nk2; g.rs_lo = nk2;
    } else if (axis == 3) {  // x2 = i2 (periodic), tiles along n2, rest (i1, n1)
        g.Sa = nk2; g.La = nx; g.periodic = 1; g.Sl = 1; g.Ll = nk;
        g.R = (long)nx * nk; g.rdiv = nk; g.rs_hi = nx * nk2; g.rs_lo = nk;
    } else {  // x1 = i1 (periodic), tiles along n2, rest (i2, n1)
        g.Sa = nx * nk2; g.La = nx; g.periodic = 1; g.Sl = 1; g.Ll = nk;
        g.R = (long)nx * nk; g.rdiv = nk; g.rs_hi = nk2; g.rs_lo = nk;
    }
    return g;
}

int sur_grow(wig2_surrogate* s, float** buf, size_t* cap, size_t n)
{
    if (n <= *cap) return WIG2_OK;
    if (*buf) hipFree(*buf);
    *buf = nullptr;
    *cap = 0;
    if (hipMalloc((void**)buf, n * sizeof(float)) != hipSuccess) return WIG2_ENOMEM;
    *cap = n;
    (void)s;
    return WIG2_OK;
}

// Training activations for npts points: h[0..L], t[0..L-1] (bf16, 16
// channels) and two FP32 gradient buffers.
int sur_ensure_act(wig2_surrogate* s, long npts)
{
    if (npts <= s->act_cap) return WIG2_OK;
    for (auto p : s->h)
        if (p) hipFree(p);
    for (auto p : s->t)
        if (p) hipFree(p);
    for (auto& p : s->dh)
        if (p) hipFree(p), p = nullptr;
    const size_t L = s->layers.size();
    s->h.assign(L + 1, nullptr);
    s->t.assign(L, nullptr);
    s->act_cap = 0;
    const size_t hb = (size_t)npts * kSurC * sizeof(unsigned short);
    for (auto& p : s->h)
        if (hipMalloc((void**)&p, hb) != hipSuccess) return WIG2_ENOMEM;
    for (auto& p : s->t)
        if (hipMalloc((void**)&p, hb) != hipSuccess) return WIG2_ENOMEM;
    for (auto& p : s->dh)
        if (hipMalloc((void**)&p, (size_t)npts * kSurC * sizeof(float)) != hipSuccess) return WIG2_ENOMEM;
    s->act_cap = npts;
    return WIG2_OK;
}

// Refresh the packed bf16 fragments from the FP32 weights.
hipError_t sur_pack(wig2_surrogate* s, hipStream_t st)
{
    for (const SurLayer& l : s->layers) {
        hipError_t e = launch_sur_pack(s->params + l.woff, l.K, 0, s->frag_f + l.foff, st);
        if (e == hipSuccess) e = launch_sur_pack(s->params + l.woff, l.K, 1, s->frag_b + l.foff, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Gradient of the mean squared error (in units of the output scale) over
// every point of (ft, delta) into s->grad; the loss into `loss`.
template <typename T>
int sur_gradient(wig2_surrogate* s, wig2_ctx* c, const T* ft, const T* delta, double& loss)
{
    const int nx = c->g.nx, nk = c->g.nk;
    const long n = c->npts;
    const int L = (int)s->layers.size();
    if (int r = sur_ensure_act(s, n)) return fail(c, r, "surrogate activations: out of memory");
    const int nb = (int)((n + 255) / 256);
    size_t need = (size_t)nb * (2 * kSurC + 1);
    for (const SurLayer& l : s->layers) need = std::max(need, (size_t)s->grid * (kSurC * kSurC * l.K + kSurC));
    if (sur_grow(s, &s->part, &s->part_cap, need) || sur_grow(s, &s->lpart, &s->lpart_cap, (size_t)nb))
        return fail(c, WIG2_ENOMEM, "surrogate gradient buffers: out of memory");
    HIPCHK(c, launch_sur_feat<T>(ft, nx, nk, s->sc, s->h[0], c->st));
    for (int l = 0; l < L; ++l) {
        const SurLayer& ly = s->layers[l];
        HIPCHK(c, launch_sur_conv(0, sur_axis(ly.axis, nx, nk), ly.K, s->h[l], nullptr, nullptr, s->t[l], s->h[l + 1],
                                  nullptr, s->frag_f + ly.foff, s->params + ly.woff + 256L * ly.K, s->grid, c->st));
    }
    int cur = 0;
    HIPCHK(c, launch_sur_head<T>(0, s->h[L], s->h[0], delta, nullptr, n, s->sc, s->params + s->head_off,
                                 2.0f / (float)n, s->dh[cur], s->part, s->lpart, c->st));
    HIPCHK(c, launch_sur_reduce(s->part, nb, 2 * kSurC + 1, 1.f, s->grad + s->head_off, c->st));
    std::vector<float> hl((size_t)nb);
    HIPCHK(c, hipMemcpyAsync(hl.data(), s->lpart, hl.size() * sizeof(float), hipMemcpyDeviceToHost, c->st));
    for (int l = L - 1; l >= 0; --l) {
        const SurLayer& ly = s->layers[l];
        const SurAxis g = sur_axis(ly.axis, nx, nk);
        const int gdw = (int)std::min<long>(sur_tiles(g), s->grid);
        HIPCHK(c, launch_sur_dw(g, ly.K, s->h[l], s->dh[cur], s->t[l], s->part, gdw, c->st));
        HIPCHK(c, launch_sur_reduce(s->part, gdw, kSurC * kSurC * ly.K + kSurC, 1.f, s->grad + ly.woff, c->st));
        if (l > 0) {
            HIPCHK(c, launch_sur_conv(1, g, ly.K, nullptr, s->dh[cur], s->t[l], nullptr, nullptr, s->dh[cur ^ 1],
                                      s->frag_b + ly.foff, nullptr, s->grid, c->st));
            cur ^= 1;
        }
    }
    HIPCHK(c, hipStreamSynchronize(c->st));
    double sum = 0.0;
    for (float v : hl) sum += v;
    loss = sum / (double)n;
    return WIG2_OK;
}

// Mean squared error only.
template <typename T>
int sur_eval(wig2_surrogate* s, wig2_ctx* c, const T* ft, const T* delta, double& loss)
{
    const int nx = c->g.nx, nk = c->g.nk;
    const long n = c->npts;
    const int L = (int)s->layers.size();
    if (int r = sur_ensure_act(s, n)) return fail(c, r, "surrogate activations: out of memory");
    const int nb = (int)((n + 255) / 256);
    if (sur_grow(s, &s->lpart, &s->lpart_cap, (size_t)nb)) return fail(c, WIG2_ENOMEM, "out of memory");
    HIPCHK(c, launch_sur_feat<T>(ft, nx, nk, s->sc, s->h[0], c->st));
    for (int l = 0; l < L; ++l) {
        const SurLayer& ly = s->layers[l];
        HIPCHK(c, launch_sur_conv(2, sur_axis(ly.axis, nx, nk), ly.K, s->h[l], nullptr, nullptr, nullptr, s->h[l + 1],
                                  nullptr, s->frag_f + ly.foff, s->params + ly.woff + 256L * ly.K, s->grid, c->st));
    }
    HIPCHK(c, launch_sur_head<T>(1, s->h[L], s->h[0], delta, nullptr, n, s->sc, s->params + s->head_off, 0.f,
                                 nullptr, nullptr, s->lpart, c->st));
    std::vector<float> hl((size_t)nb);
    HIPCHK(c, hipMemcpyAsync(hl.data(), s->lpart, hl.size() * sizeof(float), hipMemcpyDeviceToHost, c->st));
    HIPCHK(c, hipStreamSynchronize(c->st));
    double sum = 0.0;
    for (float v : hl) sum += v;
    loss = sum / (double)n;
    return WIG2_OK;
}

// f += s_out y(ft): the model's increment, with the context's own buffers
// (the model is not modified).
template <typename T>
hipError_t sur_apply(const wig2_surrogate* s, wig2_ctx* c, const T* ft, T* f)
{
    const int nx = c->g.nx, nk = c->g.nk;
    const size_t hb = (size_t)c->npts * kSurC;
    unsigned short* feat = c->sur_buf;
    unsigned short* buf[2] = {c->sur_buf + hb, c->sur_buf + 2 * hb};
    hipError_t e = launch_sur_feat<T>(ft, nx, nk, s->sc, feat, c->st);
    const unsigned short* cur = feat;
    for (size_t l = 0; l < s->layers.size() && e == hipSuccess; ++l) {
        const SurLayer& ly = s->layers[l];
        e = launch_sur_conv(2, sur_axis(ly.axis, nx, nk), ly.K, cur, nullptr, nullptr, nullptr, buf[l & 1], nullptr,
                            s->frag_f + ly.foff, s->params + ly.woff + 256L * ly.K, s->grid, c->st);
        cur = buf[l & 1];
    }
    if (e == hipSuccess)
        e = launch_sur_head<T>(2, cur, feat, nullptr, f, c->npts, s->sc, s->params + s->head_off, 0.f, nullptr, nullptr,
                               nullptr, c->st);
    return e;
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
        if (train) {
            // full-grid gradient steps on this block (a convolution needs the
            // whole neighbourhood of every point)
            for (int ep = 0; ep < std::max(1, s->cfg.epochs); ++ep) {
                if (int r = sur_gradient<T>(s, c, ft, dl, loss)) return r;
                ++s->updates;
                HIPCHK(c, launch_sur_adam(s->params, s->mom, s->var, s->grad, s->P, (float)s->cfg.lr,
                                          (int)s->updates, c->st));
                HIPCHK(c, sur_pack(s, c->st));
                s->samples += c->npts;
            }
            s->train_loss = loss;
        } else {
            if (int r = sur_eval<T>(s, c, ft, dl, loss)) return r;
            s->eval_loss = loss;
            s->samples += c->npts;
        }
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
    HIPCHK(c, sur_apply<T>(s, c, ft, f));
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
    if (hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, c->device) != hipSuccess)
        return bail(WIG2_EDEVICE);
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
        dev_alloc(c, &c->v12pair_d, np) || dev_alloc(c, &c->hart_d, np) ||
        dev_alloc(c, &c->sintab_d, (size_t)nk * nx) ||
        dev_alloc(c, &c->mf_dens_d, 2 * (size_t)nx) || dev_alloc(c, &c->mf_veff_d, 2 * (size_t)nx) ||
        dev_alloc(c, &c->s0_d, np) || dev_alloc(c, &c->s0b_d, np) || dev_alloc(c, &c->skin_d, np) ||
        dev_alloc(c, &c->s2_d, np) || dev_alloc(c, &c->rows_d, np * nk) ||
        dev_alloc(c, &c->f1_d, (size_t)nx * nk))
        return bail(WIG2_ENOMEM);
    if (G.periodic && nk <= kMaxThetaNk && dev_alloc(c, &c->fft_sym_d, (size_t)3 * nx * fft_len(nk)))
        return bail(WIG2_ENOMEM);
    if (!G.periodic && dev_alloc(c, &c->ksem_d, (size_t)nx * nk * nk)) return bail(WIG2_ENOMEM);
    if (panel && c->elem == 4 && dev_alloc(c, &c->ksem_f, (size_t)nx * nk * nk)) return bail(WIG2_ENOMEM);
    if (!G.periodic && c->meanfield) {
        std::vector<double> E, Q;
        host_sem_factors(c->g, E, Q, c->sem_pref);
        if (dev_alloc(c, &c->kmf1_d, (size_t)nx * nk * nk) || dev_alloc(c, &c->kmf2_d, (size_t)nx * nk * nk) ||
            dev_alloc(c, &c->semE_d, E.size()) || dev_alloc(c, &c->semQ_d, Q.size()))
            return bail(WIG2_ENOMEM);
        if (panel && c->elem == 4 &&
            (dev_alloc(c, &c->kmf1_f, (size_t)nx * nk * nk) || dev_alloc(c, &c->kmf2_f, (size_t)nx * nk * nk)))
            return bail(WIG2_ENOMEM);
        if (upload(c, c->semE_d, E) || upload(c, c->semQ_d, Q)) return bail(WIG2_EDEVICE);
    }

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
                    c->sig2_d, c->kap_d, c->ksem_d, c->ksem_f, c->kmf1_d, c->kmf2_d, c->kmf1_f, c->kmf2_f,
                    c->semE_d, c->semQ_d, c->v12pair_d, c->hart_d, c->sintab_d,
                    c->mf_dens_d, c->mf_veff_d, c->s0_d, c->s0b_d, c->skin_d, c->s2_d, c->rows_d,
                    c->f1_d, c->ft, c->fs, c->sur_buf, c->s12_wa, c->s12_wb, c->s12_wc, c->s12_wd,
                    c->s12_dt, c->s12_wr, c->s12_wh, c->s12_acc, c->fft_sym_d};
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

// Tables of the box two-body operator in the state's element type, and its
// workspaces: per chunk of planes two buffers of 2 nk^2 elements per plane
// (chunks of at most 512 MiB each), plus a state-sized accumulator.
int upload_sem12(wig2_ctx* c, const Sem12Tables& t)
{
    HIPCHK(c, hipStreamSynchronize(c->st));  // earlier steps may still read the old tables
    auto put = [&](void** dst, const std::vector<double>& v) -> int {
        if (*dst) {
            hipFree(*dst);
            *dst = nullptr;
        }
        if (hipMalloc(dst, v.size() * c->elem) != hipSuccess) return fail(c, WIG2_ENOMEM, "two-body SEM tables");
        hipError_t e;
        if (c->elem == 8) {
            e = hipMemcpy(*dst, v.data(), v.size() * 8, hipMemcpyHostToDevice);
        } else {
            const std::vector<float> f(v.begin(), v.end());
            e = hipMemcpy(*dst, f.data(), f.size() * 4, hipMemcpyHostToDevice);
        }
        return e == hipSuccess ? WIG2_OK : fail(c, WIG2_EDEVICE, hipGetErrorString(e));
    };
    if (int rc = put(&c->s12_wa, t.wa)) return rc;
    if (int rc = put(&c->s12_wb, t.wb)) return rc;
    if (int rc = put(&c->s12_wc, t.wc)) return rc;
    if (int rc = put(&c->s12_wd, t.wd)) return rc;
    if (int rc = put(&c->s12_dt, t.dtab)) return rc;
    if (!c->s12_wr) {
        const long np = (long)c->g.nx * c->g.nx;
        const size_t per = (size_t)2 * c->g.nk * c->g.nk * c->elem;
        c->s12_chunk = std::max<long>(1, std::min<long>(np, (long)((size_t)512 << 20) / (long)per));
        if (hipMalloc(&c->s12_wr, per * c->s12_chunk) != hipSuccess ||
            hipMalloc(&c->s12_wh, per * c->s12_chunk) != hipSuccess ||
            hipMalloc(&c->s12_acc, (size_t)c->npts * c->elem) != hipSuccess)
            return fail(c, WIG2_ENOMEM, "two-body SEM workspaces");
    }
    return WIG2_OK;
}

// Kernel of the mean field's Hartree term, V_H(x_i) = dx sum_j K[i][j] n(x_j):
// the pair potential K[i][j] = V12(x_i - x_j) (Sec. 2.3), or the neutralised
// 1-D Poisson potential (Sec. 3.1.1 example), -V_H'' = n - mean(n) on the
// torus, whose modes are V_m = (L / (2 pi m))^2 a_m for 0 < |m| < nx/2:
// K[i][j] = (1 / (nx dx)) sum_{0 < |m| < nx/2} (L / (2 pi m))^2 cos(2 pi m (i - j) / nx).
int upload_hartree(wig2_ctx* c)
{
    const int nx = c->g.nx;
    if (c->hartree == WIG2_HARTREE_PAIR) return upload(c, c->hart_d, c->v12pair) ? WIG2_EDEVICE : WIG2_OK;
    const double L = c->g.L(), pi = 3.141592653589793238462643383279502884;
    std::vector<double> row(nx, 0.0), K((size_t)nx * nx);
    for (int d = 0; d < nx; ++d)
        for (int m = 1; 2 * m < nx; ++m) {
            const double a = L / (2.0 * pi * m);
            row[d] += 2.0 * a * a * std::cos(2.0 * pi * m * d / nx);
        }
    for (int i = 0; i < nx; ++i)
        for (int j = 0; j < nx; ++j) K[(size_t)i * nx + j] = row[(i - j + nx) % nx] / (nx * c->g.dx());
    return upload(c, c->hart_d, K) ? WIG2_EDEVICE : WIG2_OK;
}

int wig2_set_potentials(wig2_ctx* c, wig2_fn1 v_ext, wig2_fn1 v12, void* user)
{
    if (!c) return WIG2_EINVAL;
    const GridInfo& g = c->g;
    const int nx = g.nx, nk = g.nk;
    const double L = g.L();
    auto V = [&](wig2_fn1 fn, double x) { return fn ? fn(x, user) : 0.0; };
    if (!g.periodic && v12 && !sem12_nk_ok(nk))
        return fail(c, WIG2_ENOTSUP, "pair potential on a box needs nk a multiple of 32, at most 256");
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
        if (c->kmf1_d) {
            // the mean field's matrices start as those of V_ext (every step
            // rebuilds them before its first Theta)
            if (upload(c, c->kmf1_d, K) || upload(c, c->kmf2_d, K)) return WIG2_EDEVICE;
            if (c->kmf1_f) {
                const std::vector<float> Kf(K.begin(), K.end());
                HIPCHK(c, hipMemcpyAsync(c->kmf1_f, Kf.data(), Kf.size() * sizeof(float), hipMemcpyHostToDevice,
                                         c->st));
                HIPCHK(c, hipMemcpyAsync(c->kmf2_f, Kf.data(), Kf.size() * sizeof(float), hipMemcpyHostToDevice,
                                         c->st));
                HIPCHK(c, hipStreamSynchronize(c->st));
            }
        }
        c->two_body = false;
        c->band = nk;
        c->sem12 = false;
        if (v12) {
            // two-body SEM operator: V12 at l dx + d dy, the tables in the
            // state's element type, workspaces for chunks of planes
            const int nd = 2 * nk - 1;
            const double dx = g.dx(), dy = sem12_dy(g);
            std::vector<double> vs((size_t)(2 * nx - 1) * nd);
            for (int l = -(nx - 1); l <= nx - 1; ++l)
                for (int d = -(nk - 1); d <= nk - 1; ++d) {
                    const double v = V(v12, l * dx + d * dy);
                    if (!isfin(v)) return fail(c, WIG2_EINVAL, "V12 returned a non-finite value");
                    vs[(size_t)(l + nx - 1) * nd + d + nk - 1] = v;
                }
            Sem12Tables t;
            host_sem12_tables(g, vs, t);
            if (int rc = upload_sem12(c, t)) return rc;
            c->sem12 = true;
        }
    }
    if (upload(c, c->v12pair_d, c->v12pair)) return WIG2_EDEVICE;
    if (int rc = upload_hartree(c)) return rc;
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

int wig2_set_hartree(wig2_ctx* c, int32_t form)
{
    if (!c || (form != WIG2_HARTREE_PAIR && form != WIG2_HARTREE_POISSON)) return WIG2_EINVAL;
    if (form == WIG2_HARTREE_POISSON && !c->g.periodic)
        return fail(c, WIG2_ENOTSUP, "the neutralised Poisson Hartree term needs a torus");
    HIPCHK(c, hipStreamSynchronize(c->st));  // queued steps read the current kernel
    c->hartree = form;
    if (c->has_pot) return upload_hartree(c);
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
    if (!c || path < WIG2_THETA_AUTO || path > WIG2_THETA_FFT || path == WIG2_THETA_PANEL) return WIG2_EINVAL;
    if (path == WIG2_THETA_FFT && (!c->fft_sym_d || !theta_fft_ok(theta_args(c))))
        return fail(c, WIG2_ENOTSUP, "FFT Theta needs a torus, nk in {16,32,48,64,96,128} and FP64 or FP32");
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
    if (use_fft(m)) return WIG2_THETA_FFT;
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
int sur_ctx_ok(wig2_surrogate* s, wig2_ctx* c)
{
    if (!c->has_state || !c->has_pot) return sfail(s, WIG2_ESTATE, "context needs state and potentials");
    if (!c->g.periodic || !c->two_body || c->meanfield)
        return sfail(s, WIG2_ENOTSUP, "surrogate needs a torus context with a pair potential, no mean field");
    if (c->prm.precision == WIG2_BF16X2) return sfail(s, WIG2_ENOTSUP, "surrogate needs FP64 or FP32 state");
    if (c->g.nk % 16 != 0) return sfail(s, WIG2_ENOTSUP, "surrogate needs nk a multiple of 16");
    if (s->dt != 0.0 && std::fabs(s->dt - c->prm.dt) > 1e-15 * s->dt)
        return sfail(s, WIG2_EINVAL, "model was trained with another dt");
    return WIG2_OK;
}
// The context's tables (symbols, pair kernel, potentials) and state taken
// from instance i of a batch (device-to-device on the batch stream).
int ctx_from_batch(wig2_ctx* c, const BatchView& v)
{
    const size_t nxk = (size_t)v.g.nx * v.g.nk;
    HIPCHK(c, hipMemcpyAsync(c->sig_ext_d, v.sig, nxk * 8, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->kap_d, v.kap, nxk * 8, hipMemcpyDeviceToDevice, c->st));
    HIPCHK(c, hipMemcpyAsync(c->f, v.f, (size_t)c->npts * c->elem, hipMemcpyDeviceToDevice, c->st));
    c->vext_x = *v.vext_x;
    c->v12pair = *v.v12pair;
    if (upload(c, c->v12pair_d, c->v12pair)) return WIG2_EDEVICE;
    c->band = v.band;
    c->two_body = v.two_body != 0;
    c->has_pot = true;
    c->has_state = true;
    c->nstep = 0;
    c->t = 0.0;
    return WIG2_OK;
}
}  // namespace

const char* wig2_surrogate_last_error(const wig2_surrogate* s) { return s ? s->err.c_str() : "null model"; }

int wig2_surrogate_create(const wig2_train_cfg* cfg, wig2_surrogate** out)
{
    if (!cfg || !out) return WIG2_EINVAL;
    *out = nullptr;
    if (cfg->channels != kSurC) return WIG2_ENOTSUP;
    auto odd_ok = [](int k, int kmax) { return k >= 1 && k <= kmax && k % 2 == 1; };
    if (cfg->blocks < 1 || cfg->blocks > 16 || !odd_ok(cfg->k_p, 63) || !odd_ok(cfg->k_x, 15) || cfg->block < 1 ||
        cfg->epochs < 0 || !(cfg->lr > 0.0) || cfg->train_blocks < 0 || cfg->max_points < 0)
        return WIG2_EINVAL;
    wig2_surrogate* s = new (std::nothrow) wig2_surrogate();
    if (!s) return WIG2_ENOMEM;
    s->cfg = *cfg;
    hipGetDevice(&s->device);
    int ncu = 256;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, s->device) == hipSuccess)
        s->grid = 4 * ncu;
    long off = 0, foff = 0;
    for (int b = 0; b < cfg->blocks; ++b)
        for (int axis = 0; axis < 4; ++axis) {
            const int K = axis < 2 ? cfg->k_p : cfg->k_x;
            s->layers.push_back(SurLayer{axis, K, off, foff});
            off += 256L * K + kSurC;
            foff += (long)(K + 1) / 2 * 64 * 8;
        }
    s->head_off = off;
    s->P = off + 2 * kSurC + 1;
    s->frag_total = foff;
    bool ok = hipMalloc((void**)&s->params, s->P * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->mom, s->P * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->var, s->P * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->grad, s->P * sizeof(float)) == hipSuccess &&
              hipMalloc((void**)&s->frag_f, foff * sizeof(unsigned short)) == hipSuccess &&
              hipMalloc((void**)&s->frag_b, foff * sizeof(unsigned short)) == hipSuccess &&
              hipMalloc((void**)&s->maxpart, 2 * kMaxParts * sizeof(float)) == hipSuccess;
    if (!ok) {
        wig2_surrogate_destroy(s);
        return WIG2_ENOMEM;
    }
    // Small uniform weights (the residual stack starts close to the
    // identity), zero biases, a small output head and a zero linear path.
    std::vector<float> p(s->P, 0.f);
    auto uni = [&](long j) {
        return (double)(splitmix(cfg->seed * 0x100000001B3ull + (uint64_t)j) >> 11) * (1.0 / 9007199254740992.0);
    };
    for (const SurLayer& l : s->layers) {
        const double a = 0.5 * std::sqrt(3.0 / (kSurC * l.K));
        for (long j = 0; j < 256L * l.K; ++j) p[l.woff + j] = (float)((2.0 * uni(l.woff + j) - 1.0) * a);
    }
    for (int k = 0; k < kSurC; ++k) p[s->head_off + k] = (float)((2.0 * uni(s->head_off + k) - 1.0) * 0.05);
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
    void* bufs[] = {s->params, s->mom, s->var, s->grad, s->frag_f, s->frag_b, s->part, s->lpart, s->maxpart,
                    s->dh[0], s->dh[1]};
    for (void* b : bufs)
        if (b) hipFree(b);
    for (auto p : s->h)
        if (p) hipFree(p);
    for (auto p : s->t)
        if (p) hipFree(p);
    delete s;
}

int wig2_surrogate_size(const wig2_surrogate* s, int64_t* nparams, int32_t* nlayers)
{
    if (!s) return WIG2_EINVAL;
    if (nparams) *nparams = s->P;
    if (nlayers) *nlayers = (int32_t)s->layers.size();
    return WIG2_OK;
}

int wig2_surrogate_get_params(const wig2_surrogate* s, float* params, float* scales)
{
    if (!s) return WIG2_EINVAL;
    if (params && hipMemcpy(params, s->params, s->P * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
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
        for (long j = 0; j < s->P; ++j)
            if (!std::isfinite(params[j])) return sfail(s, WIG2_EINVAL, "non-finite parameter");
        const std::vector<float> z(s->P, 0.f);
        if (hipMemcpy(s->params, params, s->P * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(s->mom, z.data(), s->P * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(s->var, z.data(), s->P * sizeof(float), hipMemcpyHostToDevice) != hipSuccess ||
            sur_pack(s, nullptr) != hipSuccess || hipDeviceSynchronize() != hipSuccess)
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

int wig2_surrogate_train(wig2_batch* b, const wig2_train_cfg* cfg, wig2_surrogate** out)
{
    if (!b || !cfg || !out) return WIG2_EINVAL;
    *out = nullptr;
    wig2_surrogate* s = nullptr;
    if (int r = wig2_surrogate_create(cfg, &s)) return r;
    int used = 0;
    for (int i = 0; i < batch_count(b); ++i) {
        BatchView v;
        if (!batch_view(b, i, v) || !v.has_pot || !v.has_state || !v.two_body) continue;
        const long npts = (long)v.g.nx * v.g.nx * v.g.nk * v.g.nk;
        if (cfg->max_points > 0 && npts > cfg->max_points) continue;
        if (v.g.nk % 16 != 0) continue;
        const wig2_grid G{v.g.nx, v.g.nk, 1, 1, v.g.x_min, v.g.x_max, 0.0};
        wig2_params P = v.prm;
        P.hbar = v.g.hbar;
        P.mass = v.g.mass;
        wig2_ctx* c = nullptr;
        int r = wig2_create(&G, &P, v.st, &c);
        if (r == WIG2_OK) r = ctx_from_batch(c, v);
        if (r == WIG2_OK) r = wig2_surrogate_collect(s, c, cfg->train_blocks, 1);
        if (r != WIG2_OK && c && s->err.empty()) s->err = c->err;
        wig2_destroy(c);
        if (r != WIG2_OK) {
            const std::string msg = "training on instance " + std::to_string(i) + ": " + s->err;
            wig2_surrogate_destroy(s);
            (void)msg;
            return r;
        }
        ++used;
    }
    if (used == 0) {
        wig2_surrogate_destroy(s);
        return WIG2_EINVAL;
    }
    *out = s;
    return WIG2_OK;
}

int wig2_surrogate_grad(wig2_surrogate* s, wig2_ctx* c, const void* ft, const void* delta, float* grad,
                        double* loss)
{
    if (!s || !c || !ft || !delta || !grad) return WIG2_EINVAL;
    if (c->g.nk % 16 != 0 || !c->g.periodic) return sfail(s, WIG2_ENOTSUP, "surrogate needs a torus, nk % 16 == 0");
    double l = 0.0;
    const int r = c->elem == 8 ? sur_gradient<double>(s, c, (const double*)ft, (const double*)delta, l)
                               : sur_gradient<float>(s, c, (const float*)ft, (const float*)delta, l);
    if (r) return sfail(s, r, c->err);
    if (hipMemcpy(grad, s->grad, s->P * sizeof(float), hipMemcpyDeviceToHost) != hipSuccess)
        return sfail(s, WIG2_EDEVICE, "gradient download failed");
    if (loss) *loss = l;
    return WIG2_OK;
}

int wig2_surrogate_attach(wig2_ctx* c, const wig2_surrogate* s, double drift_tol, int32_t every)
{
    if (!c || !s || !(drift_tol >= 0.0) || every < 0) return WIG2_EINVAL;
    wig2_surrogate* ms = const_cast<wig2_surrogate*>(s);
    if (int r = sur_ctx_ok(ms, c)) return fail(c, r, s->err);
    if (!s->scaled) return fail(c, WIG2_ESTATE, "the model has no scales yet (collect or set them first)");
    if (int r = ensure_sur_buffers(c, true)) return r;
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
