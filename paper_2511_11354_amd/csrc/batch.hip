// Batched ensembles of uneven periodic instances (C ABI wig2_batch_*).
//
// All instances live in three state pools (f, stage buffer, sweep buffer)
// and two FP64 symbol pools.  One Strang step covers every instance with
// two half-step sweeps, the Heun substep (two Theta stages, or the one-pass
// Heun kernel) and two half-step sweeps; within one call the last x1
// half-sweep of a step and the first of the next share one launch.
// Instances are grouped into size classes (nx, nk), heavy classes split into
// several chains of similar work; per chain and phase there is one
// persistent launch of a kernel specialised to that size (registers and LDS
// exactly as for a single grid), walking a work list of (instance, 64 lines)
// or (instance, planes) items.  Instances never interact, so each chain's
// launches are independent of the others: the HIP graphs fork one branch
// per chain (side streams during capture) and join them at the end, letting
// the device run the chains side by side.  The head, middle and tail
// segments of a call are captured once as three graphs and replayed.  Tile
// choices (planes per Theta workgroup per nk, grid sizes per class) come
// from an autotuner that times the candidates on the ensemble itself and
// keeps the winners in a small JSON cache keyed by architecture, precision
// and size class.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "common.h"

using namespace wig2;

namespace {

struct HostInst {
    GridInfo g{};
    wig2_params prm{};
    long off = 0, tab_off = 0;
    int p_off = 0;
    int band = 0, two_body = 0;
    std::vector<double> x, p, w, vext_x, v12pair;
    bool has_pot = false, has_state = false;
    long npts() const { return (long)g.nx * g.nx * g.nk * g.nk; }
};

}  // namespace

struct wig2_batch {
    int n = 0;
    int elem = 4;
    int precision = WIG2_FP32;
    std::vector<HostInst> inst;
    hipStream_t st = nullptr;
    bool own_stream = false;
    int device = 0, ncu = 256;
    std::string arch;
    long total = 0, total_tab = 0;
    int total_p = 0;
    void *f = nullptr, *k1 = nullptr, *tmp = nullptr;
    double *p_pool = nullptr, *w_pool = nullptr, *sig_pool = nullptr, *kap_pool = nullptr;
    BatchInst* insts_d = nullptr;
    AdvItem* adv_d = nullptr;
    ThItem* th_d = nullptr;
    int nadv = 0, nth = 0;
    // observables scratch (sized for the largest instance)
    double *s0 = nullptr, *skin = nullptr, *s2 = nullptr, *rows = nullptr, *f1 = nullptr;
    // tiling
    std::map<int, int> planes;  // planes per Theta workgroup, per nk
    struct Cls {
        int nx, nk;
        int th_begin, th_count, adv_begin, adv_count;
        int th_grid, adv_grid;
        bool stream;  // Theta by the streaming one-pass Heun kernel
    };
    std::vector<Cls> cls;                         // size classes (nx, nk)
    std::map<std::pair<int, int>, std::pair<int, int>> grids;  // (nx,nk) -> (theta, sweep) grid
    std::vector<hipStream_t> side;
    hipEvent_t fork = nullptr;
    std::vector<hipEvent_t> join;
    bool items_valid = false;
    hipGraph_t graph[3] = {};      // step segments: head, mid, tail
    hipGraphExec_t exec[3] = {};
    bool graph_valid = false;
    std::string err;
};

namespace {

int bfail(wig2_batch* b, int code, const std::string& m)
{
    if (b) b->err = m;
    return code;
}

#define BCHK(b, call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return bfail(b, e_ == hipErrorOutOfMemory ? WIG2_ENOMEM : WIG2_EDEVICE,     \
                         std::string(#call) + ": " + hipGetErrorString(e_));            \
    } while (0)

// Graph execs may still be running on b->st (and, through the captured
// fork/join events, on the side streams that b->st waits for).
void drop_graph(wig2_batch* b)
{
    if (b->st) hipStreamSynchronize(b->st);
    for (int k = 0; k < 3; ++k) {
        if (b->exec[k]) hipGraphExecDestroy(b->exec[k]);
        if (b->graph[k]) hipGraphDestroy(b->graph[k]);
        b->exec[k] = nullptr;
        b->graph[k] = nullptr;
    }
    b->graph_valid = false;
}

// Work lists, grouped by size class.  Theta items hold up to planes[nk]
// planes; within a class items are sorted by decreasing cost so the
// grid-stride walk balances.
int build_items(wig2_batch* b)
{
    // size classes; a class holding much more work than the average chain
    // is split into several chains so that no single chain forms a long
    // serial tail at the end of the step
    std::map<std::pair<int, int>, std::vector<int>> byshape;
    double total_work = 0.0;
    for (int i = 0; i < b->n; ++i) {
        byshape[{b->inst[i].g.nx, b->inst[i].g.nk}].push_back(i);
        total_work += (double)b->inst[i].npts() * b->inst[i].g.nk;
    }
    const double target = total_work / 24.0;
    std::vector<std::pair<std::pair<int, int>, std::vector<int>>> chains;
    for (auto& kv : byshape) {
        const double w1 = (double)b->inst[kv.second[0]].npts() * kv.first.second;
        const int per = std::max(1, (int)std::floor(target / w1));
        for (size_t a = 0; a < kv.second.size(); a += per)
            chains.push_back({kv.first, std::vector<int>(kv.second.begin() + a,
                                                         kv.second.begin() + std::min(kv.second.size(), a + per))});
    }
    std::vector<ThItem> thv;
    std::vector<AdvItem> av;
    // the work lists below are freed and rewritten: wait for launches that read them
    BCHK(b, hipStreamSynchronize(b->st));
    b->cls.clear();
    for (auto& kv : chains) {
        const int nx = kv.first.first, nk = kv.first.second;
        // a class whose instances all have a narrow single-body band takes the
        // streaming kernel (one pass per Heun step, one plane at a time),
        // exactly as a single context of that size would
        bool stream = batch_stream_nk_ok(nk, b->elem) && theta_stream_preferred(nk, b->elem);
        for (int i : kv.second) stream = stream && b->inst[i].band <= kStreamBand;
        const int P = stream ? 1 : std::max(1, std::min(b->planes[nk], batch_theta_max_planes(nk, b->elem)));
        wig2_batch::Cls c{nx, nk, (int)thv.size(), 0, (int)av.size(), 0, 4 * b->ncu, 8 * b->ncu, stream};
        if (b->grids.count(kv.first)) {
            c.th_grid = b->grids[kv.first].first;
            c.adv_grid = b->grids[kv.first].second;
        }
        const long np = (long)nx * nx, nl = (long)nx * nk * nk;
        for (int i : kv.second) {
            for (long p0 = 0; p0 < np; p0 += P)
                thv.push_back(ThItem{i, (int)p0, (int)std::min<long>(P, np - p0), 0});
            for (long l0 = 0; l0 < nl; l0 += 64) av.push_back(AdvItem{i, 0, l0});
        }
        c.th_count = (int)thv.size() - c.th_begin;
        c.adv_count = (int)av.size() - c.adv_begin;
        b->cls.push_back(c);
    }
    if (b->th_d) hipFree(b->th_d);
    if (b->adv_d) hipFree(b->adv_d);
    b->th_d = nullptr;
    b->adv_d = nullptr;
    BCHK(b, hipMalloc(&b->th_d, thv.size() * sizeof(ThItem)));
    BCHK(b, hipMalloc(&b->adv_d, av.size() * sizeof(AdvItem)));
    BCHK(b, hipMemcpyAsync(b->th_d, thv.data(), thv.size() * sizeof(ThItem), hipMemcpyHostToDevice, b->st));
    BCHK(b, hipMemcpyAsync(b->adv_d, av.data(), av.size() * sizeof(AdvItem), hipMemcpyHostToDevice, b->st));
    BCHK(b, hipStreamSynchronize(b->st));
    b->nth = (int)thv.size();
    b->nadv = (int)av.size();
    while (b->side.size() < b->cls.size()) {
        hipStream_t s2;
        BCHK(b, hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
        b->side.push_back(s2);
        hipEvent_t e;
        BCHK(b, hipEventCreateWithFlags(&e, hipEventDisableTiming));
        b->join.push_back(e);
    }
    if (!b->fork) BCHK(b, hipEventCreateWithFlags(&b->fork, hipEventDisableTiming));
    b->items_valid = true;
    drop_graph(b);
    return WIG2_OK;
}

int upload_insts(wig2_batch* b)
{
    std::vector<BatchInst> v(b->n);
    for (int i = 0; i < b->n; ++i) {
        const HostInst& h = b->inst[i];
        BatchInst& d = v[i];
        d.off = h.off;
        d.tab_off = h.tab_off;
        d.nx = h.g.nx;
        d.nk = h.g.nk;
        d.p_off = h.p_off;
        d.band = std::min(h.band, h.g.nk - 1);
        d.two_body = h.two_body;
        d.pad = 0;
        d.cpp = 0.5 * h.prm.dt / (h.g.mass * h.g.dx());
        d.tau = h.prm.dt;
    }
    // ordered after every launch already queued on b->st that reads the table
    BCHK(b, hipMemcpyAsync(b->insts_d, v.data(), v.size() * sizeof(BatchInst), hipMemcpyHostToDevice, b->st));
    BCHK(b, hipStreamSynchronize(b->st));
    drop_graph(b);
    return WIG2_OK;
}

template <typename T>
hipError_t class_advect(wig2_batch* b, const wig2_batch::Cls& c, int dim, const void* in, void* out,
                        int grid, hipStream_t st, int passes = 1)
{
    return launch_advect_batch<T>((const T*)in, (T*)out, b->insts_d, b->adv_d + c.adv_begin, c.adv_count,
                                  dim, b->p_pool, c.nx, grid, st, passes);
}

template <typename T>
hipError_t class_theta(wig2_batch* b, const wig2_batch::Cls& c, int mode, const void* u, const void* v,
                       void* out, int grid, hipStream_t st)
{
    return launch_theta_batch<T>((const T*)u, (const T*)v, (T*)out, b->insts_d, b->th_d + c.th_begin,
                                 c.th_count, mode, b->sig_pool, b->kap_pool, c.nk, b->planes[c.nk], grid, st);
}

// The Heun sub-step of one size class on pool `f` (k1 as stage buffer).
template <typename T>
hipError_t class_heun(wig2_batch* b, const wig2_batch::Cls& c, void* f, int grid, hipStream_t st)
{
    if (c.stream)
        return launch_theta_stream_batch<T>((T*)f, b->insts_d, b->th_d + c.th_begin, c.th_count, b->sig_pool,
                                            b->kap_pool, c.nk, grid, st);
    hipError_t e = class_theta<T>(b, c, 0, f, nullptr, b->k1, grid, st);
    return e != hipSuccess ? e : class_theta<T>(b, c, 1, f, b->k1, f, grid, st);
}

// Strang steps of one size class, in the sweep order of a single context's
// multi-step call: a step enters with the x1 then x2 half-sweeps and leaves
// with x2 then x1, and between two steps of one call the two x1 half-sweeps
// run as one two-pass launch.  A call of n steps is
//   head (x1 f->tmp, x2 tmp->f, Heun f, x2 f->tmp)
//   n - 1 times mid (x1 x1 tmp->k1, x2 k1->f, Heun f, x2 f->tmp)
//   tail (x1 tmp->f),
// so every segment starts and ends in the same pools (k1, the general
// Heun's stage buffer, is free between Heun stages).
enum Seg { SEG_HEAD = 0, SEG_MID = 1, SEG_TAIL = 2 };

template <typename T>
hipError_t class_seg(wig2_batch* b, const wig2_batch::Cls& c, int seg, hipStream_t st)
{
    hipError_t e;
    if (seg == SEG_TAIL) return class_advect<T>(b, c, 1, b->tmp, b->f, c.adv_grid, st);
    if (seg == SEG_HEAD) {
        if ((e = class_advect<T>(b, c, 1, b->f, b->tmp, c.adv_grid, st)) != hipSuccess) return e;
        if ((e = class_advect<T>(b, c, 2, b->tmp, b->f, c.adv_grid, st)) != hipSuccess) return e;
    } else {
        if ((e = class_advect<T>(b, c, 1, b->tmp, b->k1, c.adv_grid, st, 2)) != hipSuccess) return e;
        if ((e = class_advect<T>(b, c, 2, b->k1, b->f, c.adv_grid, st)) != hipSuccess) return e;
    }
    if ((e = class_heun<T>(b, c, b->f, c.th_grid, st)) != hipSuccess) return e;
    return class_advect<T>(b, c, 2, b->f, b->tmp, c.adv_grid, st);
}

// One segment for every class: one chain per class, forked from and joined
// back to the batch stream (parallel branches under capture).
template <typename T>
hipError_t enqueue_seg(wig2_batch* b, int seg)
{
    if (b->cls.size() == 1) return class_seg<T>(b, b->cls[0], seg, b->st);
    hipError_t e = hipEventRecord(b->fork, b->st);
    if (e != hipSuccess) return e;
    for (size_t c = 0; c < b->cls.size(); ++c) {
        if ((e = hipStreamWaitEvent(b->side[c], b->fork, 0)) != hipSuccess) return e;
        if ((e = class_seg<T>(b, b->cls[c], seg, b->side[c])) != hipSuccess) return e;
        if ((e = hipEventRecord(b->join[c], b->side[c])) != hipSuccess) return e;
    }
    for (size_t c = 0; c < b->cls.size(); ++c)
        if ((e = hipStreamWaitEvent(b->st, b->join[c], 0)) != hipSuccess) return e;
    return hipSuccess;
}

// One whole step (head then tail).
template <typename T>
hipError_t enqueue_step(wig2_batch* b)
{
    hipError_t e = enqueue_seg<T>(b, SEG_HEAD);
    return e != hipSuccess ? e : enqueue_seg<T>(b, SEG_TAIL);
}

// Runs one step directly (kernel attributes are set by uncaptured launches
// first; the joint x1 launch needs none), then captures the three segments.
int capture(wig2_batch* b)
{
    if (!b->items_valid && build_items(b)) return WIG2_EDEVICE;
    drop_graph(b);
    hipError_t e = b->elem == 8 ? enqueue_step<double>(b) : enqueue_step<float>(b);
    if (e != hipSuccess) return bfail(b, WIG2_EDEVICE, std::string("batch step: ") + hipGetErrorString(e));
    BCHK(b, hipStreamSynchronize(b->st));
    for (int seg = 0; seg < 3; ++seg) {
        BCHK(b, hipStreamBeginCapture(b->st, hipStreamCaptureModeGlobal));
        e = b->elem == 8 ? enqueue_seg<double>(b, seg) : enqueue_seg<float>(b, seg);
        hipGraph_t g = nullptr;
        hipError_t e2 = hipStreamEndCapture(b->st, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) hipGraphDestroy(g);
            drop_graph(b);
            return bfail(b, WIG2_EDEVICE, "graph capture failed");
        }
        b->graph[seg] = g;
        BCHK(b, hipGraphInstantiate(&b->exec[seg], g, nullptr, nullptr, 0));
    }
    b->graph_valid = true;
    return WIG2_OK;
}

// ---- autotuner cache (tiny flat JSON: {"key": value, ...}) -----------------

std::map<std::string, int> read_cache(const std::string& path)
{
    std::map<std::string, int> m;
    std::ifstream in(path);
    if (!in) return m;
    std::stringstream ss;
    ss << in.rdbuf();
    const std::string s = ss.str();
    size_t pos = 0;
    while ((pos = s.find('"', pos)) != std::string::npos) {
        const size_t e = s.find('"', pos + 1);
        if (e == std::string::npos) break;
        const std::string key = s.substr(pos + 1, e - pos - 1);
        size_t c = s.find(':', e);
        if (c == std::string::npos) break;
        m[key] = std::atoi(s.c_str() + c + 1);
        pos = s.find_first_of(",}", c);
        if (pos == std::string::npos) break;
    }
    return m;
}

void write_cache(const std::string& path, const std::map<std::string, int>& m)
{
    std::ofstream out(path);
    out << "{";
    bool first = true;
    for (auto& kv : m) {
        out << (first ? "" : ",") << "\n  \"" << kv.first << "\": " << kv.second;
        first = false;
    }
    out << "\n}\n";
}

std::string key_prefix(const wig2_batch* b)
{
    return b->arch + (b->elem == 8 ? "/fp64" : "/fp32");
}

template <typename F>
float time_ms(wig2_batch* b, F&& launch, int reps)
{
    hipEvent_t a, c;
    hipEventCreate(&a);
    hipEventCreate(&c);
    launch();  // warm
    hipEventRecord(a, b->st);
    for (int r = 0; r < reps; ++r) launch();
    hipEventRecord(c, b->st);
    hipEventSynchronize(c);
    float ms = 0.f;
    hipEventElapsedTime(&ms, a, c);
    hipEventDestroy(a);
    hipEventDestroy(c);
    return ms / reps;
}

}  // namespace

extern "C" {

int wig2_batch_create(int32_t n, const wig2_grid* grids, const wig2_params* params, void* stream,
                      wig2_batch** out)
{
    if (!out || n <= 0 || !grids || !params) return WIG2_EINVAL;
    *out = nullptr;
    const int prec = params[0].precision;
    for (int i = 0; i < n; ++i) {
        const wig2_grid& G = grids[i];
        const wig2_params& P = params[i];
        if (G.nx < 4 || G.nk < 2 || !(G.x_max > G.x_min) || !std::isfinite(G.x_min) ||
            !std::isfinite(G.x_max) || !(P.hbar > 0) || !(P.mass > 0) || !(P.dt > 0) ||
            !std::isfinite(P.dt) || !std::isfinite(P.hbar) || !std::isfinite(P.mass))
            return WIG2_EINVAL;
        if (P.precision != prec || (prec != WIG2_FP32 && prec != WIG2_FP64)) return WIG2_ENOTSUP;
        if (!G.periodic || P.scheme != WIG2_STRANG || P.meanfield_lambda != 0.0 || P.xc)
            return WIG2_ENOTSUP;
        if (!batch_nx_ok(G.nx) || !batch_nk_ok(G.nk)) return WIG2_ENOTSUP;
        const double L = G.x_max - G.x_min, dx = L / G.nx;
        const double pmax = P.hbar * 3.141592653589793 / L * (G.nk / 2);
        if (0.5 * P.dt * pmax / (P.mass * dx) > 1.0) return WIG2_ENOTSUP;
    }
    wig2_batch* b = new (std::nothrow) wig2_batch();
    if (!b) return WIG2_ENOMEM;
    auto bail = [&](int code) {
        wig2_batch_destroy(b);
        return code;
    };
    b->n = n;
    b->precision = prec;
    b->elem = prec == WIG2_FP64 ? 8 : 4;
    b->inst.resize(n);
    long off = 0, toff = 0;
    int poff = 0, maxnx = 0, maxnk = 0;
    long maxpts = 0;
    for (int i = 0; i < n; ++i) {
        HostInst& h = b->inst[i];
        h.g = GridInfo{grids[i].nx, grids[i].nk, 1, 1, grids[i].x_min, grids[i].x_max, 0.0,
                       params[i].hbar, params[i].mass};
        h.prm = params[i];
        h.off = off;
        h.tab_off = toff;
        h.p_off = poff;
        off += h.npts();
        toff += (long)h.g.nx * h.g.nk;
        poff += h.g.nk;
        maxnx = std::max(maxnx, h.g.nx);
        maxnk = std::max(maxnk, h.g.nk);
        maxpts = std::max(maxpts, h.npts());
        host_nodes(h.g, h.x, h.p, h.w);
    }
    b->total = off;
    b->total_tab = toff;
    b->total_p = poff;
    if (hipGetDevice(&b->device) != hipSuccess) return bail(WIG2_EDEVICE);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) return bail(WIG2_EDEVICE);
    b->ncu = prop.multiProcessorCount;
    b->arch = prop.gcnArchName;
    {
        const size_t c = b->arch.find(':');
        if (c != std::string::npos) b->arch = b->arch.substr(0, c);
    }
    for (int k : {16, 32, 48, 64, 96, 128})
        b->planes[k] = std::max(1, std::min(8 / std::max(1, k / 16), batch_theta_max_planes(k, b->elem)));
    if (stream) {
        b->st = static_cast<hipStream_t>(stream);
    } else {
        if (hipStreamCreateWithFlags(&b->st, hipStreamNonBlocking) != hipSuccess) return bail(WIG2_EDEVICE);
        b->own_stream = true;
    }
    const size_t bytes = (size_t)b->total * b->elem;
    if (hipMalloc(&b->f, bytes) != hipSuccess || hipMalloc(&b->k1, bytes) != hipSuccess ||
        hipMalloc(&b->tmp, bytes) != hipSuccess)
        return bail(WIG2_ENOMEM);
    if (hipMalloc(&b->p_pool, sizeof(double) * poff) != hipSuccess ||
        hipMalloc(&b->w_pool, sizeof(double) * poff) != hipSuccess ||
        hipMalloc(&b->sig_pool, sizeof(double) * toff) != hipSuccess ||
        hipMalloc(&b->kap_pool, sizeof(double) * toff) != hipSuccess ||
        hipMalloc(&b->insts_d, sizeof(BatchInst) * n) != hipSuccess)
        return bail(WIG2_ENOMEM);
    const size_t np = (size_t)maxnx * maxnx;
    if (hipMalloc(&b->s0, np * 8) != hipSuccess || hipMalloc(&b->skin, np * 8) != hipSuccess ||
        hipMalloc(&b->s2, np * 8) != hipSuccess || hipMalloc(&b->rows, np * maxnk * 8) != hipSuccess ||
        hipMalloc(&b->f1, (size_t)maxnx * maxnk * 8) != hipSuccess)
        return bail(WIG2_ENOMEM);
    std::vector<double> pp(poff), ww(poff), zero(toff, 0.0);
    for (int i = 0; i < n; ++i) {
        std::copy(b->inst[i].p.begin(), b->inst[i].p.end(), pp.begin() + b->inst[i].p_off);
        std::copy(b->inst[i].w.begin(), b->inst[i].w.end(), ww.begin() + b->inst[i].p_off);
    }
    if (hipMemcpy(b->p_pool, pp.data(), poff * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->w_pool, ww.data(), poff * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->sig_pool, zero.data(), toff * 8, hipMemcpyHostToDevice) != hipSuccess ||
        hipMemcpy(b->kap_pool, zero.data(), toff * 8, hipMemcpyHostToDevice) != hipSuccess)
        return bail(WIG2_EDEVICE);
    if (upload_insts(b)) return bail(WIG2_EDEVICE);
    *out = b;
    return WIG2_OK;
}

void wig2_batch_destroy(wig2_batch* b)
{
    if (!b) return;
    if (b->st) hipStreamSynchronize(b->st);
    drop_graph(b);
    for (hipStream_t s2 : b->side) hipStreamDestroy(s2);
    for (hipEvent_t e : b->join) hipEventDestroy(e);
    if (b->fork) hipEventDestroy(b->fork);
    void* bufs[] = {b->f, b->k1, b->tmp, b->p_pool, b->w_pool, b->sig_pool, b->kap_pool, b->insts_d,
                    b->adv_d, b->th_d, b->s0, b->skin, b->s2, b->rows, b->f1};
    for (void* p : bufs)
        if (p) hipFree(p);
    if (b->own_stream && b->st) hipStreamDestroy(b->st);
    delete b;
}

const char* wig2_batch_last_error(const wig2_batch* b) { return b ? b->err.c_str() : "null batch"; }

int wig2_batch_set_potentials(wig2_batch* b, int32_t i, wig2_fn1 v_ext, wig2_fn1 v12, void* user)
{
    if (!b || i < 0 || i >= b->n) return WIG2_EINVAL;
    HostInst& h = b->inst[i];
    const GridInfo& g = h.g;
    const int nx = g.nx, nk = g.nk;
    const double L = g.L();
    auto V = [&](wig2_fn1 fn, double x) { return fn ? fn(x, user) : 0.0; };
    std::vector<double> vy(2 * nk), vr(2 * nk), s, vh, kap;
    for (int j = 0; j < 2 * nk; ++j) {
        vy[j] = V(v_ext, g.x_min + L * j / (2 * nk));
        vr[j] = V(v12, -0.5 * L + L * j / (2 * nk));
        if (!std::isfinite(vy[j]) || !std::isfinite(vr[j])) return bfail(b, WIG2_EINVAL, "non-finite potential");
    }
    host_symbol_ext(g, vy, s);
    host_pair_kernel(g, vr, vh, kap);
    double smax = 0.0;
    for (double v : s) smax = std::max(smax, std::fabs(v));
    h.band = 0;
    for (int m = 1; m < nk; ++m)
        for (int x = 0; x < nx; ++x)
            if (std::fabs(s[(size_t)x * nk + m]) > 1e-13 * smax) h.band = std::max(h.band, m);
    h.two_body = 0;
    for (int m = 1; m < nk; ++m)
        if (vh[m] != 0.0) h.two_body = 1;
    h.vext_x.resize(nx);
    for (int k = 0; k < nx; ++k) h.vext_x[k] = V(v_ext, h.x[k]);
    h.v12pair.assign((size_t)nx * nx, 0.0);
    for (int a = 0; a < nx; ++a)
        for (int c = 0; c < nx; ++c) {
            double r = h.x[a] - h.x[c];
            r -= L * std::floor((r + 0.5 * L) / L);
            h.v12pair[(size_t)a * nx + c] = V(v12, r);
        }
    BCHK(b, hipMemcpyAsync(b->sig_pool + h.tab_off, s.data(), s.size() * 8, hipMemcpyHostToDevice, b->st));
    BCHK(b, hipMemcpyAsync(b->kap_pool + h.tab_off, kap.data(), kap.size() * 8, hipMemcpyHostToDevice, b->st));
    BCHK(b, hipStreamSynchronize(b->st));
    h.has_pot = true;
    return upload_insts(b);
}

}  // extern "C"

namespace wig2 {
int batch_count(const wig2_batch* b) { return b ? b->n : 0; }
bool batch_view(const wig2_batch* b, int i, BatchView& v)
{
    if (!b || i < 0 || i >= b->n) return false;
    const HostInst& h = b->inst[i];
    v.g = h.g;
    v.prm = h.prm;
    v.elem = b->elem;
    v.f = static_cast<const char*>(b->f) + (size_t)h.off * b->elem;
    v.sig = b->sig_pool + h.tab_off;
    v.kap = b->kap_pool + h.tab_off;
    v.band = h.band;
    v.two_body = h.two_body;
    v.vext_x = &h.vext_x;
    v.v12pair = &h.v12pair;
    v.has_pot = h.has_pot;
    v.has_state = h.has_state;
    v.st = b->st;
    return true;
}
}  // namespace wig2

extern "C" {

int wig2_batch_set_state(wig2_batch* b, int32_t i, const double* fh)
{
    if (!b || !fh || i < 0 || i >= b->n) return WIG2_EINVAL;
    HostInst& h = b->inst[i];
    // on b->st, after the steps still in flight that read or write the pool
    if (b->elem == 8) {
        BCHK(b, hipMemcpyAsync((double*)b->f + h.off, fh, h.npts() * 8, hipMemcpyHostToDevice, b->st));
        BCHK(b, hipStreamSynchronize(b->st));
    } else {
        std::vector<float> t(h.npts());
        for (long k = 0; k < h.npts(); ++k) t[k] = (float)fh[k];
        BCHK(b, hipMemcpyAsync((float*)b->f + h.off, t.data(), h.npts() * 4, hipMemcpyHostToDevice, b->st));
        BCHK(b, hipStreamSynchronize(b->st));
    }
    h.has_state = true;
    return WIG2_OK;
}

int wig2_batch_get_state(wig2_batch* b, int32_t i, double* fh)
{
    if (!b || !fh || i < 0 || i >= b->n) return WIG2_EINVAL;
    HostInst& h = b->inst[i];
    BCHK(b, hipStreamSynchronize(b->st));
    if (b->elem == 8) {
        BCHK(b, hipMemcpyAsync(fh, (double*)b->f + h.off, h.npts() * 8, hipMemcpyDeviceToHost, b->st));
        BCHK(b, hipStreamSynchronize(b->st));
    } else {
        std::vector<float> t(h.npts());
        BCHK(b, hipMemcpyAsync(t.data(), (float*)b->f + h.off, h.npts() * 4, hipMemcpyDeviceToHost, b->st));
        BCHK(b, hipStreamSynchronize(b->st));
        for (long k = 0; k < h.npts(); ++k) fh[k] = t[k];
    }
    return WIG2_OK;
}

int wig2_batch_step(wig2_batch* b, int64_t nsteps)
{
    if (!b || nsteps < 0) return WIG2_EINVAL;
    for (auto& h : b->inst)
        if (!h.has_pot || !h.has_state) return bfail(b, WIG2_ESTATE, "every instance needs potentials and a state");
    if (nsteps == 0) return WIG2_OK;
    if (!b->graph_valid) {
        int rc = capture(b);
        if (rc) return rc;
        --nsteps;  // the capture pass ran one step directly
        if (nsteps == 0) return WIG2_OK;
    }
    BCHK(b, hipGraphLaunch(b->exec[SEG_HEAD], b->st));
    for (int64_t s = 1; s < nsteps; ++s) BCHK(b, hipGraphLaunch(b->exec[SEG_MID], b->st));
    BCHK(b, hipGraphLaunch(b->exec[SEG_TAIL], b->st));
    return WIG2_OK;
}

int wig2_batch_observables(wig2_batch* b, int32_t i, wig2_obs* o, double* n1, double* n12, double* f1)
{
    if (!b || !o || i < 0 || i >= b->n) return WIG2_EINVAL;
    HostInst& h = b->inst[i];
    const int nx = h.g.nx, nk = h.g.nk;
    const size_t np = (size_t)nx * nx;
    hipError_t e = b->elem == 8
                       ? launch_plane_moments<double>((const double*)b->f + h.off, nx, nk, b->p_pool + h.p_off,
                                                      b->w_pool + h.p_off, 0.5 / h.g.mass, b->s0, b->skin,
                                                      b->s2, b->rows, b->st)
                       : launch_plane_moments<float>((const float*)b->f + h.off, nx, nk, b->p_pool + h.p_off,
                                                     b->w_pool + h.p_off, 0.5 / h.g.mass, b->s0, b->skin,
                                                     b->s2, b->rows, b->st);
    if (e != hipSuccess) return bfail(b, WIG2_EDEVICE, hipGetErrorString(e));
    const double dx = h.g.dx();
    BCHK(b, launch_reduce_rows(b->rows, nx, nk, dx, b->f1, b->st));
    std::vector<double> s0(np), sk(np), s2(np), hf1((size_t)nx * nk);
    BCHK(b, hipMemcpyAsync(s0.data(), b->s0, np * 8, hipMemcpyDeviceToHost, b->st));
    BCHK(b, hipMemcpyAsync(sk.data(), b->skin, np * 8, hipMemcpyDeviceToHost, b->st));
    BCHK(b, hipMemcpyAsync(s2.data(), b->s2, np * 8, hipMemcpyDeviceToHost, b->st));
    BCHK(b, hipMemcpyAsync(hf1.data(), b->f1, hf1.size() * 8, hipMemcpyDeviceToHost, b->st));
    BCHK(b, hipStreamSynchronize(b->st));
    double mass = 0, en = 0, l2 = 0;
    for (int a = 0; a < nx; ++a)
        for (int c = 0; c < nx; ++c) {
            const size_t q = (size_t)a * nx + c;
            const double vp = (h.vext_x.empty() ? 0.0 : h.vext_x[a] + h.vext_x[c]) +
                              (h.v12pair.empty() ? 0.0 : h.v12pair[q]);
            mass += s0[q];
            en += sk[q] + vp * s0[q];
            l2 += s2[q];
        }
    o->step = 0;
    o->t = 0.0;
    o->mass = dx * dx * mass;
    o->energy = dx * dx * en;
    o->l2 = dx * dx * l2;
    std::vector<double> occ;
    o->entropy_vn = host_entropy(h.g, hf1, occ);
    o->fallbacks = 0;
    if (n12) std::copy(s0.begin(), s0.end(), n12);
    if (n1)
        for (int a = 0; a < nx; ++a) {
            double s = 0;
            for (int c = 0; c < nx; ++c) s += s0[(size_t)a * nx + c];
            n1[a] = dx * s;
        }
    if (f1) std::copy(hf1.begin(), hf1.end(), f1);
    if (!std::isfinite(o->mass) || !std::isfinite(o->energy)) return bfail(b, WIG2_ENUMERIC, "non-finite observable");
    return WIG2_OK;
}

int wig2_batch_info(const wig2_batch* b, int64_t* total_points, int32_t* theta_grid, int32_t* advect_grid,
                    int32_t* planes_per_group)
{
    if (!b) return WIG2_EINVAL;
    if (total_points) *total_points = b->total;
    int k = 0;
    for (int c : {16, 32, 48, 64, 96, 128}) {
        int tg = 0, ag = 0;
        for (auto& cl : b->cls) {
            if (cl.nk == c) tg = std::max(tg, cl.th_grid);
            if (cl.nx == c) ag = std::max(ag, cl.adv_grid);
        }
        if (theta_grid) theta_grid[k] = tg;
        if (advect_grid) advect_grid[k] = ag;
        if (planes_per_group) planes_per_group[k] = b->planes.at(c);
        ++k;
    }
    return WIG2_OK;
}

int wig2_batch_tune(wig2_batch* b, const char* cache_path, int32_t force)
{
    if (!b) return WIG2_EINVAL;
    for (auto& h : b->inst)
        if (!h.has_pot || !h.has_state) return bfail(b, WIG2_ESTATE, "tune after potentials and states are set");
    if (build_items(b)) return WIG2_EDEVICE;
    const std::string pre = key_prefix(b);
    std::map<std::string, int> cache;
    if (cache_path && *cache_path) cache = read_cache(cache_path);
    auto kp = [&](int nk) { return pre + "/theta/nk" + std::to_string(nk) + "/planes"; };
    // Theta grids are kept per kernel (streaming or general) of the class
    auto kc = [&](const wig2_batch::Cls& c, const char* what) {
        const std::string kind = std::string(what) == "theta" ? (c.stream ? "stream/" : "general/") : "";
        return pre + "/" + what + "/" + kind + "nx" + std::to_string(c.nx) + "nk" + std::to_string(c.nk) + "/grid";
    };
    bool have = !force;
    for (auto& c : b->cls)
        have = have && cache.count(kp(c.nk)) && cache.count(kc(c, "theta")) && cache.count(kc(c, "advect"));
    if (have) {
        for (auto& c : b->cls) {
            b->planes[c.nk] = cache[kp(c.nk)];
            b->grids[{c.nx, c.nk}] = {cache[kc(c, "theta")], cache[kc(c, "advect")]};
        }
        return build_items(b);
    }
    // the state is read-only input while tuning: copy it to the sweep buffer
    const size_t bytes = (size_t)b->total * b->elem;
    BCHK(b, hipMemcpyAsync(b->tmp, b->f, bytes, hipMemcpyDeviceToDevice, b->st));
    auto t_adv = [&](const wig2_batch::Cls& c, int grid) {
        return time_ms(b, [&] {
            b->elem == 8 ? class_advect<double>(b, c, 2, b->tmp, b->k1, grid, b->st)
                         : class_advect<float>(b, c, 2, b->tmp, b->k1, grid, b->st);
        }, 3);
    };
    auto t_th = [&](const wig2_batch::Cls& c, int grid) {
        return time_ms(b, [&] {
            b->elem == 8 ? class_heun<double>(b, c, b->tmp, grid, b->st) : class_heun<float>(b, c, b->tmp, grid, b->st);
        }, 2);
    };
    // 1. planes per Theta workgroup per nk, timed over all classes of that nk
    std::vector<int> nks;
    for (auto& c : b->cls)
        if (std::find(nks.begin(), nks.end(), c.nk) == nks.end()) nks.push_back(c.nk);
    for (int nk : nks) {
        bool stream_nk = false;
        for (auto& c : b->cls)
            if (c.nk == nk && c.stream) stream_nk = true;
        if (stream_nk) continue;  // one plane at a time
        const int maxp = std::max(1, std::min(4, batch_theta_max_planes(nk, b->elem)));
        float best = 1e30f;
        int bp = b->planes[nk];
        for (int P = 1; P <= maxp; ++P) {
            b->planes[nk] = P;
            if (build_items(b)) return WIG2_EDEVICE;
            float t = 0.f;
            for (auto& c : b->cls)
                if (c.nk == nk) t += t_th(c, c.th_grid);
            if (t < best) { best = t; bp = P; }
        }
        b->planes[nk] = bp;
    }
    if (build_items(b)) return WIG2_EDEVICE;
    // 2. grid sizes per class (the first chain of each (nx, nk) stands for all)
    std::map<std::pair<int, int>, bool> done;
    for (auto& c : b->cls) {
        if (done[{c.nx, c.nk}]) continue;
        done[{c.nx, c.nk}] = true;
        float best = 1e30f;
        int bt = c.th_grid, ba = c.adv_grid;
        for (int m : {1, 2, 4, 8, 16}) {
            const float t = t_th(c, m * b->ncu);
            if (t < best) { best = t; bt = m * b->ncu; }
        }
        best = 1e30f;
        for (int m : {1, 2, 4, 8, 16, 32}) {
            const float t = t_adv(c, m * b->ncu);
            if (t < best) { best = t; ba = m * b->ncu; }
        }
        b->grids[{c.nx, c.nk}] = {bt, ba};
    }
    BCHK(b, hipStreamSynchronize(b->st));
    if (build_items(b)) return WIG2_EDEVICE;
    // 3. whole step with all classes running together: the grids tuned one
    //    class at a time against one workgroup per item (the hardware then
    //    spreads the concurrent classes); keep the faster.
    {
        void* keep = nullptr;
        BCHK(b, hipMalloc(&keep, bytes));
        BCHK(b, hipMemcpyAsync(keep, b->f, bytes, hipMemcpyDeviceToDevice, b->st));
        auto t_step = [&] {
            return time_ms(b, [&] { b->elem == 8 ? enqueue_step<double>(b) : enqueue_step<float>(b); }, 2);
        };
        const float t_tuned = t_step();
        const auto tuned = b->grids;
        for (auto& c : b->cls) b->grids[{c.nx, c.nk}] = {c.th_count, (c.adv_count + 3) / 4};
        if (build_items(b)) return WIG2_EDEVICE;
        const float t_items = t_step();
        if (!(t_items < t_tuned)) {
            b->grids = tuned;
            if (build_items(b)) return WIG2_EDEVICE;
        }
        BCHK(b, hipMemcpyAsync(b->f, keep, bytes, hipMemcpyDeviceToDevice, b->st));
        BCHK(b, hipStreamSynchronize(b->st));
        hipFree(keep);
    }
    for (auto& c : b->cls) {
        cache[kp(c.nk)] = b->planes[c.nk];
        cache[kc(c, "theta")] = c.th_grid;
        cache[kc(c, "advect")] = c.adv_grid;
    }
    if (cache_path && *cache_path) write_cache(cache_path, cache);
    return WIG2_OK;
}

}  // extern "C"
