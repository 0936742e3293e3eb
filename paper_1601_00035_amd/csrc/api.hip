// C-ABI of the library: handle lifecycle, per-box convolution plans (LGF spectrum, twiddles,
// workspaces), the integrating factor, the IF-HERK stage driver and Vor2Vel.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <iterator>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "kernels.h"

namespace nslgf {

static thread_local std::string g_last_error;
void set_error(const std::string& msg) { g_last_error = msg; }

// Device buffer that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
    int ensure(size_t need) {
        if (need <= bytes) return NSLGF_OK;
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        if (hipMalloc(&p, need) != hipSuccess) {
            (void)hipGetLastError();
            set_error("hipMalloc of " + std::to_string(need) + " bytes failed");
            return NSLGF_ENOMEM;
        }
        bytes = need;
        return NSLGF_OK;
    }
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
};

struct ConvPlan {
    int nx = 0, ny = 0, nz = 0, dtype = 0;
    int Px = 0, Py = 0, Pz = 0;
    long long XP = 0;
    int tb = 0, tiles = 0;
    int vy = 0, vz = 0;  // column-pass plan variants of the y and z lengths
    DevBuf khat;
    DevBuf A1, A2;  // workspaces for up to 3 components
};

}  // namespace nslgf

namespace nslgf {
// Event pairs around kernel launches, resolved lazily.
struct Profiler {
    bool on = false;
    struct Rec {
        std::string name;
        hipEvent_t a, b;
    };
    std::vector<Rec> pending;
    std::vector<hipEvent_t> pool;
    std::map<std::string, std::pair<long long, double>> totals;
    std::vector<std::string> order;
    hipEvent_t get() {
        if (!pool.empty()) {
            hipEvent_t e = pool.back();
            pool.pop_back();
            return e;
        }
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        return e;
    }
    void resolve() {
        for (auto& r : pending) {
            float ms = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
                auto it = totals.find(r.name);
                if (it == totals.end()) {
                    order.push_back(r.name);
                    it = totals.emplace(r.name, std::make_pair(0LL, 0.0)).first;
                }
                it->second.first += 1;
                it->second.second += ms;
            }
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        pending.clear();
    }
    ~Profiler() {
        for (auto& r : pending) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};
}  // namespace nslgf

namespace nslgf {
// The launch tuner's record of one box and dtype: the launch shapes (once tuned or loaded) and the
// column-plan variants (-1 until a tuned or loaded plan sets them).
struct TuneEntry {
    Tuning t;
    bool launch_set = false;
    int vy = -1, vz = -1;
};

// One captured batch step, reused while the batch (boxes, pointers, step parameters) is unchanged.
struct BatchGraph {
    std::vector<unsigned long long> key;
    hipGraphExec_t exec = nullptr;
    DevBuf desc;       // argument tables of the batched passes (read by the graph's kernels)
    int groups = 0;    // groups of problems run as batched passes (0: one branch of kernels per problem)
    int launches = 0;  // kernel launches in the graph
    ~BatchGraph() {
        if (exec) (void)hipGraphExecDestroy(exec);
    }
};
}  // namespace nslgf

struct nslgf_ctx {
    int device = 0;
    nslgf::Profiler prof;
    std::unique_ptr<nslgf::BatchGraph> batch;
    std::vector<hipStream_t> branches;
    std::vector<hipEvent_t> batch_events;
    hipStream_t capture = nullptr;
    ~nslgf_ctx() {
        for (auto s : branches) (void)hipStreamDestroy(s);
        for (auto e : batch_events) (void)hipEventDestroy(e);
        if (capture) (void)hipStreamDestroy(capture);
    }
    bool capturing = false;  // a batch graph is being captured (no host round trips)
    int batch_mode = NSLGF_BATCH_PASSES;
    bool no_alloc = false;   // inside lgf_convolve_noalloc: lookups that would allocate fail instead
    void* scratch = nullptr; // this device's address of the library's fixed scratch array
    int fft_plan = -1;  // column-pass plan choice: -1 per-dtype default, -2 autotune, else a variant index
    int tune_mode = NSLGF_TUNE_DEFAULT;
    // launch shapes per (nx, ny, nz, dtype): tuned on first use in NSLGF_TUNE_AUTO, or loaded from a file
    std::map<std::tuple<int, int, int, int>, nslgf::TuneEntry> tunings;
    std::map<std::tuple<int, int, int, int, int>, std::unique_ptr<nslgf::ConvPlan>> plans;
    std::map<std::pair<int, int>, std::unique_ptr<nslgf::DevBuf>> twiddles;  // (L, dtype)
    nslgf::DevBuf if_tmp1, if_tmp2, tmp3, tmp3b, partial, blockmask;
    nslgf::DevBuf act_u[2], act_d, act_w, act_work, act_mask;  // the active-box driver's box state
};

namespace nslgf {

// Fixed device scratch of the allocation-free convolution: each device that loads the library holds
// its own copy for the life of the process.  Host code never passes the array's name to a kernel (it
// is a host-side stand-in there); it uses the device address taken by hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[NSLGF_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_addr;  // device -> address of `scratch` on that device

// Address of `scratch` on the current device `device` (taken once per device).
static int scratch_address(int device, void** out) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_addr.find(device);
    if (it == g_scratch_addr.end()) {
        void* ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || ptr == nullptr) {
            set_error(std::string("hipGetSymbolAddress of the scratch array failed: ") + hipGetErrorString(e));
            return NSLGF_EHIP;
        }
        it = g_scratch_addr.emplace(device, ptr).first;
    }
    *out = it->second;
    return NSLGF_OK;
}

static int get_twiddles(nslgf_ctx* h, int L, int dtype, const void** out) {
    auto key = std::make_pair(L, dtype);
    auto it = h->twiddles.find(key);
    if (it == h->twiddles.end() && h->no_alloc) {
        set_error("lgf_convolve_noalloc: no twiddle table for this box and dtype; call lgf_table first");
        return NSLGF_ESTATE;
    }
    if (it == h->twiddles.end()) {
        void* d = nullptr;
        NSLGF_TRY(make_twiddles(L, dtype, &d));
        auto b = std::make_unique<DevBuf>();
        b->p = d;
        b->bytes = (size_t)L * 2 * dtype_size(dtype);
        it = h->twiddles.emplace(key, std::move(b)).first;
    }
    *out = it->second->p;
    return NSLGF_OK;
}

// Brackets one launch with profiling events when collection is on.
struct ProfScope {
    nslgf_ctx* h;
    const char* name;
    hipStream_t s;
    hipEvent_t a = nullptr;
    ProfScope(nslgf_ctx* h_, const char* n, hipStream_t s_) : h(h_), name(n), s(s_) {
        if (h && h->prof.on) {
            a = h->prof.get();
            if (a) (void)hipEventRecord(a, s);
        }
    }
    ~ProfScope() {
        if (a) {
            hipEvent_t b = h->prof.get();
            if (b) {
                (void)hipEventRecord(b, s);
                h->prof.pending.push_back({name, a, b});
            } else {
                h->prof.pool.push_back(a);
            }
        }
    }
};
#define NSLGF_PROF(h, name, s, expr)                                                               \
    do {                                                                                           \
        ProfScope ps_(h, name, s);                                                                 \
        NSLGF_TRY(expr);                                                                           \
    } while (0)

static int check_box(int nx, int ny, int nz) {
    NSLGF_CHECK_ARG(nx >= 1 && ny >= 1 && nz >= 1 && nx <= 256 && ny <= 256 && nz <= 256,
                    "box sizes must be in 1..256 per axis");
    return NSLGF_OK;
}

static int check_dtype(int dtype) {
    NSLGF_CHECK_ARG(dtype == NSLGF_F64 || dtype == NSLGF_F32, "dtype must be NSLGF_F64 or NSLGF_F32");
    return NSLGF_OK;
}

static int padded(int n) {
    // smallest supported even length P >= 2n - 1
    return next_supported_length(2 * n - 1 > 16 ? 2 * n - 1 : 16);
}

// Five-pass convolution of ncomp scalar fields with a plan's spectrum times `scale`.
// Source given as the masked divergence of a 3-component face field (formed by the first pass).
struct DivSource {
    const void* f;
    int nbuf;
    double idx;
    const unsigned char* blocks = nullptr;  // support blocks (replace the nbuf rule when set)
    int nb = 0;
};
static int run_conv(nslgf_ctx* h, ConvPlan& p, const void* src, void* dst, int ncomp, double scale, hipStream_t s,
                    void* A1, void* A2, const DivSource* div = nullptr);
// Twiddle tables of a plan's lengths for a dtype (built on first use; call before any capture).
static int plan_twiddles(nslgf_ctx* h, const ConvPlan& p, int dt, const void** twh, const void** twf, const void** twy,
                         const void** twz);

// Timing of one launch sequence: the minimum over `reps` runs (after one warm-up run) of the
// event-to-event time on the stream, in milliseconds.
template <class F> static int time_min_ms(hipStream_t s, int reps, F&& run, float* best) {
    hipEvent_t a = nullptr, b = nullptr;
    NSLGF_HIP_CHECK(hipEventCreate(&a));
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        set_error("hipEventCreate failed");
        return NSLGF_EHIP;
    }
    int rc = run();
    *best = 3.4e38f;
    for (int i = 0; rc == NSLGF_OK && i < reps; ++i) {
        float ms = 0.f;
        if (hipEventRecord(a, s) != hipSuccess) rc = NSLGF_EHIP;
        if (rc == NSLGF_OK) rc = run();
        if (rc == NSLGF_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                               hipEventElapsedTime(&ms, a, b) != hipSuccess))
            rc = NSLGF_EHIP;
        if (rc == NSLGF_OK) *best = std::min(*best, ms);
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (rc == NSLGF_EHIP) set_error("autotune: event timing failed");
    return rc;
}

// The tuners' rule: every candidate is timed (minimum of 5 runs after a warm-up) and replaces the
// default only when it is at least 3 % faster, so that timing noise between near-equal choices does not
// move a choice away from the measured default.
template <class C, class F> static int pick_fastest(hipStream_t s, C deflt, std::initializer_list<C> cands, F&& run,
                                                    C* out) {
    float tdef = 0.f;
    NSLGF_TRY(time_min_ms(s, 5, [&] { return run(deflt); }, &tdef));
    C best = deflt;
    float tbest = tdef;
    for (C c : cands) {
        if (c == deflt) continue;
        float ms = 0.f;
        NSLGF_TRY(time_min_ms(s, 5, [&] { return run(c); }, &ms));
        if (ms < 0.97f * tdef && ms < tbest) {
            tbest = ms;
            best = c;
        }
    }
    *out = best;
    return NSLGF_OK;
}

// Autotuner of the column-pass plans: times every variant that exists for the plan's y and z lengths
// on the plan's own shapes (one component, zero data, the workspaces of one solve) and keeps the
// fastest for each.  Runs once per plan, before any capture.
static int autotune_plan(nslgf_ctx* h, ConvPlan& p, hipStream_t s) {
    const int dt = p.dtype;
    const size_t es = dtype_size(dt);
    DevBuf a1, a2;
    NSLGF_TRY(a1.ensure((size_t)p.nz * p.ny * p.XP * 2 * es));
    NSLGF_TRY(a2.ensure((size_t)p.nz * p.Py * p.XP * 2 * es));
    NSLGF_HIP_CHECK(hipMemsetAsync(a1.p, 0, a1.bytes, s));
    NSLGF_HIP_CHECK(hipMemsetAsync(a2.p, 0, a2.bytes, s));
    const void *twy, *twz;
    NSLGF_TRY(get_twiddles(h, p.Py, dt, &twy));
    NSLGF_TRY(get_twiddles(h, p.Pz, dt, &twz));
    ColPass y{};
    y.ncols = p.Px / 2 + 1;
    y.nouter = p.nz;
    y.in_row = y.out_row = p.XP;
    y.ncomp = 1;
    y.tw = twy;
    ColPass z{};
    z.in = z.out = a2.p;
    z.ncols = p.Px / 2 + 1;
    z.nouter = p.Py;
    z.in_outer = z.out_outer = p.XP;
    z.in_row = z.out_row = (long long)p.Py * p.XP;
    z.ncomp = 1;
    z.n_in = z.n_out = p.nz;
    z.tw = twz;
    z.khat = p.khat.p;
    z.khat_tiles = p.tiles;
    z.outer_period = p.Py;
    z.scale = 1.0;
    auto valid = [&](int L, std::initializer_list<int> all) {
        std::vector<int> v;
        for (int x : all)
            if (col_variant_valid(L, dt, x)) v.push_back(x);
        return v;
    };
    {
        int best = p.vz;
        const std::vector<int> vs = valid(p.Pz, {0, 1, 2});
        float tdef = 0.f;
        NSLGF_TRY(time_min_ms(s, 5, [&] { return launch_col(p.Pz, dt, COL_CONV, z, s, p.vz); }, &tdef));
        float tbest = tdef;
        for (int v : vs) {
            if (v == p.vz) continue;
            float ms = 0.f;
            NSLGF_TRY(time_min_ms(s, 5, [&] { return launch_col(p.Pz, dt, COL_CONV, z, s, v); }, &ms));
            if (ms < 0.97f * tdef && ms < tbest) {
                tbest = ms;
                best = v;
            }
        }
        p.vz = best;
    }
    {
        auto run = [&](int v) {
            ColPass f = y, b = y;
            f.in = a1.p;
            f.out = a2.p;
            f.in_outer = (long long)p.ny * p.XP;
            f.out_outer = (long long)p.Py * p.XP;
            f.n_in = p.ny;
            f.n_out = p.Py;
            b.in = a2.p;
            b.out = a1.p;
            b.in_outer = (long long)p.Py * p.XP;
            b.out_outer = (long long)p.ny * p.XP;
            b.n_in = p.Py;
            b.n_out = p.ny;
            const int rc = launch_col(p.Py, dt, COL_FWD, f, s, v);
            return rc != NSLGF_OK ? rc : launch_col(p.Py, dt, COL_INV, b, s, v);
        };
        int best = p.vy;
        const std::vector<int> vs = valid(p.Py, {0, 1, 2});
        float tdef = 0.f;
        NSLGF_TRY(time_min_ms(s, 5, [&] { return run(p.vy); }, &tdef));
        float tbest = tdef;
        for (int v : vs) {
            if (v == p.vy) continue;
            float ms = 0.f;
            NSLGF_TRY(time_min_ms(s, 5, [&] { return run(v); }, &ms));
            if (ms < 0.97f * tdef && ms < tbest) {
                tbest = ms;
                best = v;
            }
        }
        p.vy = best;
    }
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    return NSLGF_OK;
}

static int build_plan(nslgf_ctx* h, int nx, int ny, int nz, int dtype, hipStream_t s, ConvPlan** out) {
    auto key = std::make_tuple(nx, ny, nz, dtype, h->fft_plan);
    auto it = h->plans.find(key);
    if (it != h->plans.end()) {
        *out = it->second.get();
        return NSLGF_OK;
    }
    // (a plan is built, never recorded: its launches run even inside a recording)
    struct Unrecord {
        LaunchRecorder* r = launch_recorder();
        Unrecord() { launch_recorder() = nullptr; }
        ~Unrecord() { launch_recorder() = r; }
    } unrecord;
    auto plan = std::make_unique<ConvPlan>();
    ConvPlan& p = *plan;
    p.nx = nx;
    p.ny = ny;
    p.nz = nz;
    p.dtype = dtype;
    p.Px = padded(nx);
    p.Py = padded(ny);
    p.Pz = padded(nz);
    if (p.Px < 0 || p.Py < 0 || p.Pz < 0) {
        set_error("no supported padded length for this box");
        return NSLGF_EUNSUPPORTED;
    }
    p.XP = ((p.Px / 2 + 1 + 7) / 8) * 8;
    p.vy = col_variant_choice(p.Py, dtype, h->fft_plan, false);
    p.vz = col_variant_choice(p.Pz, dtype, h->fft_plan, true);
    auto te = h->tunings.find(std::make_tuple(nx, ny, nz, dtype));
    const bool loaded = h->fft_plan == -1 && te != h->tunings.end() && te->second.vy >= 0 && te->second.vz >= 0 &&
                        col_variant_valid(p.Py, dtype, te->second.vy) && col_variant_valid(p.Pz, dtype, te->second.vz);
    if (loaded) {  // a tuned choice recorded for this box (by the tuner or from a tuning file)
        p.vy = te->second.vy;
        p.vz = te->second.vz;
    }
    p.tb = col_tile_width(p.Pz, dtype);
    p.tiles = ceil_div(p.Px / 2 + 1, p.tb);
    // FP64 kernel on the padded lattice and its spectrum
    const long long ktot = (long long)p.Px * p.Py * p.Pz;
    DevBuf kr, spec;
    NSLGF_TRY(kr.ensure(ktot * sizeof(double)));
    NSLGF_TRY(spec.ensure((size_t)p.Pz * p.Py * p.XP * 2 * sizeof(double)));
    NSLGF_TRY(build_padded_lgf(p.Px, p.Py, p.Pz, (double*)kr.p, s));
    const void *twh, *twf, *twy, *twz;
    NSLGF_TRY(get_twiddles(h, p.Px / 2, NSLGF_F64, &twh));
    NSLGF_TRY(get_twiddles(h, p.Px, NSLGF_F64, &twf));
    NSLGF_TRY(get_twiddles(h, p.Py, NSLGF_F64, &twy));
    NSLGF_TRY(get_twiddles(h, p.Pz, NSLGF_F64, &twz));
    RowPass r{};
    r.in = kr.p;
    r.out = spec.p;
    r.nrows = (long long)p.Pz * p.Py;
    r.in_row = p.Px;
    r.out_row = p.XP;
    r.ncomp = 1;
    r.n_io = p.Px;
    r.tw_half = twh;
    r.tw_full = twf;
    NSLGF_TRY(launch_row_r2c(p.Px, NSLGF_F64, r, s));
    ColPass c{};
    c.in = spec.p;
    c.out = spec.p;
    c.ncols = p.Px / 2 + 1;
    c.nouter = p.Pz;
    c.in_outer = c.out_outer = (long long)p.Py * p.XP;
    c.in_row = c.out_row = p.XP;
    c.ncomp = 1;
    c.n_in = c.n_out = p.Py;
    c.tw = twy;
    NSLGF_TRY(launch_col(p.Py, NSLGF_F64, COL_FWD, c, s));
    c.nouter = p.Py;
    c.in_outer = c.out_outer = p.XP;
    c.in_row = c.out_row = (long long)p.Py * p.XP;
    c.n_in = c.n_out = p.Pz;
    c.tw = twz;
    NSLGF_TRY(launch_col(p.Pz, NSLGF_F64, COL_FWD, c, s));
    const size_t kbytes = (size_t)(p.Py / 2 + 1) * p.tiles * (p.Pz / 2 + 1) * p.tb * dtype_size(dtype);
    NSLGF_TRY(p.khat.ensure(kbytes));
    NSLGF_TRY(extract_spectrum(spec.p, p.Px, p.Py, p.Pz, p.XP, 1.0 / (double)ktot, p.tb, p.tiles, dtype, p.khat.p, s));
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    if (h->fft_plan == NSLGF_FFT_PLAN_AUTOTUNE || (h->tune_mode == NSLGF_TUNE_AUTO && !loaded && h->fft_plan == -1)) {
        NSLGF_TRY(autotune_plan(h, p, s));
        if (h->fft_plan == -1) {
            TuneEntry& e = h->tunings[std::make_tuple(nx, ny, nz, dtype)];
            e.vy = p.vy;
            e.vz = p.vz;
        }
    }
    *out = plan.get();
    h->plans.emplace(key, std::move(plan));
    return NSLGF_OK;
}

static int plan_twiddles(nslgf_ctx* h, const ConvPlan& p, int dt, const void** twh, const void** twf, const void** twy,
                         const void** twz) {
    NSLGF_TRY(get_twiddles(h, p.Px / 2, dt, twh));
    NSLGF_TRY(get_twiddles(h, p.Px, dt, twf));
    NSLGF_TRY(get_twiddles(h, p.Py, dt, twy));
    NSLGF_TRY(get_twiddles(h, p.Pz, dt, twz));
    return NSLGF_OK;
}

// Default launch shapes of a box, the tuner's choices on cubes of 48 to 256 cells: output rows per
// workgroup of the fused x-y integrating-factor pass 32 up to 128 cells along y, 64 up to 192, else 128
// (small planes give few workgroups, each a serial walk over its rows: shorter walks, more of them);
// outputs per thread of the strided z pass 16 up to 192 cells along z, else 32.
static Tuning default_tuning(int nx, int ny, int nz) {
    (void)nx;
    Tuning t;
    t.if_rows = ny <= 128 ? 32 : ny <= 192 ? 64 : 128;
    t.if_seg = nz <= 192 ? 16 : 32;
    return t;
}

// Launch tuner: times, on zero fields of the box, the fused x-y integrating-factor pass for 32, 64, 128
// and 256 rows per workgroup, the strided z pass for 16 and 32 outputs per thread, and the stage kernel
// (the largest point kernel) for every point-kernel shape, and keeps the fastest of each.  None of
// these choices changes the arithmetic.  Runs once per box and dtype, outside any capture.
static int autotune_launch(nslgf_ctx* h, int nx, int ny, int nz, int dtype, hipStream_t s, Tuning* out) {
    const size_t f3 = (size_t)3 * nx * ny * nz * dtype_size(dtype);
    DevBuf a, b, c, d;
    NSLGF_TRY(a.ensure(f3));
    NSLGF_TRY(b.ensure(f3));
    NSLGF_TRY(c.ensure(f3));
    NSLGF_TRY(d.ensure(f3));
    for (DevBuf* x : {&a, &b, &c, &d}) NSLGF_HIP_CHECK(hipMemsetAsync(x->p, 0, x->bytes, s));
    double w[kIfMaxRadius + 1];
    const int rad = if_weights(0.02, dtype, w, kIfMaxRadius);  // the step's typical factor (beta / 2)
    const bool prof = h->prof.on;
    h->prof.on = false;
    Tuning t = default_tuning(nx, ny, nz);
    int rc = NSLGF_OK;
    {
        const IfCombine cb{{a.p, nullptr, nullptr}, {1.0, 0.0, 0.0}};
        // (more rows than half the plane gives one tile: the same launch as fewer rows would)
        std::initializer_list<int> rows_all = {32, 64, 128, 256};
        std::vector<int> rows_ok;
        for (int r : rows_all)
            if (r <= 32 || ny > r / 2) rows_ok.push_back(r);
        int best = t.if_rows;
        float tdef = 0.f;
        rc = time_min_ms(s, 5, [&] { return launch_if_xy(dtype, cb, b.p, 3, nx, ny, nz, w, rad, s, t.if_rows); }, &tdef);
        float tbest = tdef;
        for (int r : rows_ok) {
            if (rc != NSLGF_OK || r == t.if_rows) continue;
            float ms = 0.f;
            rc = time_min_ms(s, 5, [&] { return launch_if_xy(dtype, cb, b.p, 3, nx, ny, nz, w, rad, s, r); }, &ms);
            if (rc == NSLGF_OK && ms < 0.97f * tdef && ms < tbest) {
                tbest = ms;
                best = r;
            }
        }
        t.if_rows = best;
    }
    if (rc == NSLGF_OK)
        rc = pick_fastest(s, t.if_seg, {32, 16}, [&](int seg) {
            return launch_if_axis(2, dtype, b.p, a.p, 3, nx, ny, nz, w, rad, s, seg);
        }, &t.if_seg);
    if (rc == NSLGF_OK) {
        StageCoef cf{};
        cf.c_q = 1.0;
        cf.c_w1 = 0.5;
        cf.c_g = -0.5;
        rc = pick_fastest(s, t.cell_shape, {0, 1, 2, 3}, [&](int shape) {
            return launch_stage_rhs(dtype, a.p, b.p, c.p, nullptr, d.p, cf, nx, ny, nz, 1.0, s, shape);
        }, &t.cell_shape);
    }
    h->prof.on = prof;
    NSLGF_TRY(rc);
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    *out = t;
    return NSLGF_OK;
}

// Launch shapes for a box and dtype: a tuned or loaded entry, else (in NSLGF_TUNE_AUTO, outside a
// capture) tuned now, else the defaults.
static int get_tuning(nslgf_ctx* h, int nx, int ny, int nz, int dtype, hipStream_t s, Tuning* out) {
    auto key = std::make_tuple(nx, ny, nz, dtype);
    auto it = h->tunings.find(key);
    if (it != h->tunings.end() && it->second.launch_set) {
        *out = it->second.t;
        return NSLGF_OK;
    }
    if (h->tune_mode == NSLGF_TUNE_AUTO && !h->capturing && !h->no_alloc) {
        Tuning t;
        NSLGF_TRY(autotune_launch(h, nx, ny, nz, dtype, s, &t));
        TuneEntry& e = h->tunings[key];
        e.t = t;
        e.launch_set = true;
        *out = t;
        return NSLGF_OK;
    }
    *out = default_tuning(nx, ny, nz);
    return NSLGF_OK;
}

// Workspaces of one convolution of up to 3 components: A1 [nz][ny][XP] and A2 [nz][Py][XP] complex.
static size_t conv_ws_elems_a1(const ConvPlan& p) { return (size_t)p.nz * p.ny * p.XP * 2; }
static size_t conv_ws_elems_a2(const ConvPlan& p) { return (size_t)p.nz * p.Py * p.XP * 2; }

static int run_conv(nslgf_ctx* h, ConvPlan& p, const void* src, void* dst, int ncomp, double scale, hipStream_t s,
                    void* A1, void* A2, const DivSource* div) {
    const int dt = p.dtype;
    const long long a1c = (long long)p.nz * p.ny * p.XP, a2c = (long long)p.nz * p.Py * p.XP;
    const void *twh, *twf, *twy, *twz;
    NSLGF_TRY(plan_twiddles(h, p, dt, &twh, &twf, &twy, &twz));
    const long long box = (long long)p.nx * p.ny * p.nz;
    RowPass r{};
    r.in = src;
    r.out = A1;
    r.nrows = (long long)p.nz * p.ny;
    r.in_row = p.nx;
    r.out_row = p.XP;
    r.in_comp = box;
    r.out_comp = a1c;
    r.ncomp = ncomp;
    r.n_io = p.nx;
    r.tw_half = twh;
    r.tw_full = twf;
    if (div) {
        if (ncomp != 1) {
            set_error("run_conv: a divergence source has one component");
            return NSLGF_EINVAL;
        }
        r.div_src = div->f;
        r.div_ny = p.ny;
        r.div_nz = p.nz;
        r.div_nbuf = div->nbuf;
        r.div_idx = div->idx;
        r.div_blocks = div->blocks;
        r.div_nb = div->nb;
    }
    NSLGF_PROF(h, "conv_x_r2c", s, launch_row_r2c(p.Px, dt, r, s));
    ColPass c{};
    c.in = A1;
    c.out = A2;
    c.ncols = p.Px / 2 + 1;
    c.nouter = p.nz;
    c.in_outer = (long long)p.ny * p.XP;
    c.out_outer = (long long)p.Py * p.XP;
    c.in_row = c.out_row = p.XP;
    c.in_comp = a1c;
    c.out_comp = a2c;
    c.ncomp = ncomp;
    c.n_in = p.ny;
    c.n_out = p.Py;
    c.tw = twy;
    NSLGF_PROF(h, "conv_y_fwd", s, launch_col(p.Py, dt, COL_FWD, c, s, p.vy));
    ColPass z{};
    z.in = A2;
    z.out = A2;
    z.ncols = p.Px / 2 + 1;
    z.nouter = p.Py;
    z.in_outer = z.out_outer = p.XP;
    z.in_row = z.out_row = (long long)p.Py * p.XP;
    z.in_comp = z.out_comp = a2c;
    z.ncomp = ncomp;
    z.n_in = z.n_out = p.nz;
    z.tw = twz;
    z.khat = p.khat.p;
    z.khat_tiles = p.tiles;
    z.outer_period = p.Py;
    z.scale = scale;
    NSLGF_PROF(h, "conv_z_fused", s, launch_col(p.Pz, dt, COL_CONV, z, s, p.vz));
    ColPass y{};
    y.in = A2;
    y.out = A1;
    y.ncols = p.Px / 2 + 1;
    y.nouter = p.nz;
    y.in_outer = (long long)p.Py * p.XP;
    y.out_outer = (long long)p.ny * p.XP;
    y.in_row = y.out_row = p.XP;
    y.in_comp = a2c;
    y.out_comp = a1c;
    y.ncomp = ncomp;
    y.n_in = p.Py;
    y.n_out = p.ny;
    y.tw = twy;
    NSLGF_PROF(h, "conv_y_inv", s, launch_col(p.Py, dt, COL_INV, y, s, p.vy));
    RowPass o{};
    o.in = A1;
    o.out = dst;
    o.nrows = (long long)p.nz * p.ny;
    o.in_row = p.XP;
    o.out_row = p.nx;
    o.in_comp = a1c;
    o.out_comp = box;
    o.ncomp = ncomp;
    o.n_io = p.nx;
    o.tw_half = twh;
    o.tw_full = twf;
    NSLGF_PROF(h, "conv_x_c2r", s, launch_row_c2r(p.Px, dt, o, s));
    return NSLGF_OK;
}

// Convolution on the plan's own workspaces (handle-level calls; not for concurrent streams).
static int run_conv_shared(nslgf_ctx* h, ConvPlan& p, const void* src, void* dst, int ncomp, double scale,
                           hipStream_t s) {
    const size_t es = dtype_size(p.dtype);
    NSLGF_TRY(p.A1.ensure(3 * conv_ws_elems_a1(p) * es));
    NSLGF_TRY(p.A2.ensure(3 * conv_ws_elems_a2(p) * es));
    return run_conv(h, p, src, dst, ncomp, scale, s, p.A1.p, p.A2.p);
}

// IF application through two temporaries (x: src -> t1, y: t1 -> t2, z: t2 -> dst); src == dst allowed.
static int run_if(nslgf_ctx* h, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double alpha, int dtype,
                  hipStream_t s, void* t1, void* t2, const Tuning& tn) {
    const long long n = (long long)nx * ny * nz;
    if (alpha == 0.0) {
        // identity: an elementwise kernel copy (no memory-copy nodes when the caller captures a graph)
        if (src != dst)
            NSLGF_PROF(h, "copy", s, launch_axpby(dtype, dst, src, 1.0, nullptr, 0.0, nullptr, 0.0, ncomp * n, s));
        return NSLGF_OK;
    }
    double w[kIfMaxRadius + 1];
    const int r = if_weights(alpha, dtype, w, kIfMaxRadius);
    if (r < 0) return NSLGF_EINVAL;
    if (r >= 1 && r <= kIfFixedMaxRadius) {
        const IfCombine cb{{src, nullptr, nullptr}, {1.0, 0.0, 0.0}};
        NSLGF_PROF(h, "if_xy", s, launch_if_xy(dtype, cb, t1, ncomp, nx, ny, nz, w, r, s, tn.if_rows));
        NSLGF_PROF(h, "if_z", s, launch_if_axis(2, dtype, t1, dst, ncomp, nx, ny, nz, w, r, s, tn.if_seg));
        return NSLGF_OK;
    }
    NSLGF_PROF(h, "if_x", s, launch_if_axis(0, dtype, src, t1, ncomp, nx, ny, nz, w, r, s));
    NSLGF_PROF(h, "if_y", s, launch_if_axis(1, dtype, t1, t2, ncomp, nx, ny, nz, w, r, s));
    NSLGF_PROF(h, "if_z", s, launch_if_axis(2, dtype, t2, dst, ncomp, nx, ny, nz, w, r, s));
    return NSLGF_OK;
}

// M E(alpha) M applied to the combination c0 p0 + c1 p1 + c2 p2 (formed in FP64, rounded once): the
// combination is formed while the fused x-y pass loads its input, so it never makes a round trip
// through memory; identity and runtime-radius cases combine first into dst.
static int run_if_combined(nslgf_ctx* h, const IfCombine& cb, void* dst, int ncomp, int nx, int ny, int nz,
                           double alpha, int dtype, hipStream_t s, void* t1, void* t2, const Tuning& tn) {
    const long long n = (long long)nx * ny * nz;
    if (alpha != 0.0) {
        double w[kIfMaxRadius + 1];
        const int r = if_weights(alpha, dtype, w, kIfMaxRadius);
        if (r < 0) return NSLGF_EINVAL;
        if (r >= 1 && r <= kIfFixedMaxRadius) {
            NSLGF_PROF(h, "if_xy", s, launch_if_xy(dtype, cb, t1, ncomp, nx, ny, nz, w, r, s, tn.if_rows));
            NSLGF_PROF(h, "if_z", s, launch_if_axis(2, dtype, t1, dst, ncomp, nx, ny, nz, w, r, s, tn.if_seg));
            return NSLGF_OK;
        }
    }
    NSLGF_PROF(h, "axpby", s,
               launch_axpby(dtype, dst, cb.p[0], cb.c[0], cb.p[1], cb.c[1], cb.p[2], cb.c[2], ncomp * n, s));
    return run_if(h, dst, dst, ncomp, nx, ny, nz, alpha, dtype, s, t1, t2, tn);
}

// u = M E(alpha) M (r - G dhat) with the stage's w update, the projection formed while the fused x-y
// pass loads (r - G dhat never makes a round trip through memory); alpha = 0 or runtime radii project
// first into r.
static int run_if_projected(nslgf_ctx* h, void* r, const IfProject& pj, void* dst, int nx, int ny, int nz,
                            double alpha, int dtype, double dx, hipStream_t s, void* t1, void* t2, const Tuning& tn) {
    if (alpha != 0.0) {
        double w[kIfMaxRadius + 1];
        const int rad = if_weights(alpha, dtype, w, kIfMaxRadius);
        if (rad < 0) return NSLGF_EINVAL;
        if (rad >= 1 && rad <= kIfFixedMaxRadius && nx <= 256) {
            IfCombine cb{{r, nullptr, nullptr}, {1.0, 0.0, 0.0}};
            cb.proj = &pj;
            NSLGF_PROF(h, "if_xy", s, launch_if_xy(dtype, cb, t1, 3, nx, ny, nz, w, rad, s, tn.if_rows));
            NSLGF_PROF(h, "if_z", s, launch_if_axis(2, dtype, t1, dst, 3, nx, ny, nz, w, rad, s, tn.if_seg));
            return NSLGF_OK;
        }
    }
    void* proj_out = alpha == 0.0 ? dst : r;
    NSLGF_PROF(h, "stage_project", s,
               launch_stage_project(dtype, r, proj_out, pj.dhat, pj.q, pj.w1, nullptr, pj.c_q, pj.c_w1, 0.0, pj.wnew,
                                    pj.inv, nx, ny, nz, dx, s, tn.cell_shape));
    if (alpha != 0.0) NSLGF_TRY(run_if(h, r, dst, 3, nx, ny, nz, alpha, dtype, s, t1, t2, tn));
    return NSLGF_OK;
}

static int run_if_shared(nslgf_ctx* h, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double alpha,
                         int dtype, hipStream_t s, const Tuning& tn) {
    const size_t bytes = (size_t)ncomp * nx * ny * nz * dtype_size(dtype);
    NSLGF_TRY(h->if_tmp1.ensure(bytes));
    NSLGF_TRY(h->if_tmp2.ensure(bytes));
    return run_if(h, src, dst, ncomp, nx, ny, nz, alpha, dtype, s, h->if_tmp1.p, h->if_tmp2.p, tn);
}

// Layout of an IF-HERK state's workspace, in elements of its dtype.
struct StateLayout {
    size_t q, w1, w2, r, dhat, t1, t2, a1, a2, total;
};
static StateLayout state_layout(int nx, int ny, int nz) {
    const size_t M = (size_t)nx * ny * nz;
    const int Py = padded(ny);
    const int Px = padded(nx);
    const size_t XP = (size_t)(((Px / 2 + 1 + 7) / 8) * 8);
    StateLayout L{};
    L.q = 0;
    L.w1 = 3 * M;   // w1 directly after q: stage 2 applies H^1 to both as one 6-component field
    L.w2 = 6 * M;
    L.r = 9 * M;
    L.dhat = 12 * M;  // (the pressure source is formed inside the convolution's first pass)
    L.t1 = 13 * M;    // IF temporaries, 6 components each
    L.t2 = 19 * M;
    L.a1 = 25 * M;    // one-component convolution workspaces (complex)
    L.a2 = L.a1 + (size_t)nz * ny * XP * 2;
    L.total = L.a2 + (size_t)nz * Py * XP * 2;
    return L;
}

// The step guard's two accumulators (FP64 divergence maximum, non-finite count) sit after the workspace.
constexpr size_t kGuardBytes = 256;
static size_t state_guard_offset(int nx, int ny, int nz, int dtype) {
    const size_t b = state_layout(nx, ny, nz).total * dtype_size(dtype);
    return (b + 255) / 256 * 256;
}

// Shifted tableau a~, c~ (1-based, c~_0 = 0) of the three-stage schemes (Sec. 3.1, 3.2).
static void tableau(int scheme, double at[4][4], double ct[4]) {
    const double s3 = std::sqrt(3.0);
    double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}}, b[3], c[3];
    if (scheme == NSLGF_SCHEME_B) {
        A[1][0] = 1.0 / 3.0;
        A[2][0] = -1.0;
        A[2][1] = 2.0;
        b[0] = 0.0; b[1] = 0.75; b[2] = 0.25;
        c[0] = 0.0; c[1] = 1.0 / 3.0; c[2] = 1.0;
    } else if (scheme == NSLGF_SCHEME_C) {
        A[1][0] = 8.0 / 15.0;
        A[2][0] = 0.25;
        A[2][1] = 5.0 / 12.0;
        b[0] = 0.25; b[1] = 0.0; b[2] = 0.75;
        c[0] = 0.0; c[1] = 8.0 / 15.0; c[2] = 2.0 / 3.0;
    } else {
        A[1][0] = 0.5;
        A[2][0] = s3 / 3.0;
        A[2][1] = (3.0 - s3) / 3.0;
        b[0] = (3.0 + s3) / 6.0; b[1] = -s3 / 3.0; b[2] = (3.0 + s3) / 6.0;
        c[0] = 0.0; c[1] = 0.5; c[2] = 1.0;
    }
    std::memset(at, 0, sizeof(double) * 16);
    ct[0] = 0.0;
    for (int i = 1; i <= 3; ++i) {
        for (int j = 1; j <= 3; ++j) at[i][j] = (i < 3) ? A[i][j - 1] : b[j - 1];
        ct[i] = (i < 3) ? c[i] : 1.0;
    }
}

// Records one step of every state (no launch), groups the states whose launch records match position
// by position (same kernels, grids and blocks: boxes of one size, dtype, scheme and integrating-factor
// radii), and captures one graph in which every position of every group is one launch over a table of
// the group's arguments, the groups on their own branch streams.  NSLGF_ESTATE if some step has a
// launch without a batched form (nothing captured).  Plans, twiddles and launch shapes exist already.
static int capture_batched_passes(nslgf_ctx* h, nslgf_state* const* sts, int n, hipStream_t s,
                                  const std::vector<unsigned long long>& key) {
    std::vector<LaunchRecorder> recs(n);
    bool ok = true;
    const bool prof_was = h->prof.on;
    h->prof.on = false;
    h->capturing = true;  // (no host round trips while recording)
    for (int i = 0; i < n && ok; ++i) {
        const nslgf_state saved = *sts[i];
        launch_recorder() = &recs[i];
        const int rc = ::herk_step(h, sts[i], s);
        launch_recorder() = nullptr;
        *sts[i] = saved;
        if (rc != NSLGF_OK) {
            h->capturing = false;
            h->prof.on = prof_was;
            return rc;
        }
        ok = recs[i].ok;
    }
    h->capturing = false;
    h->prof.on = prof_was;
    if (!ok) return NSLGF_ESTATE;
    auto same = [](const LaunchRecorder& a, const LaunchRecorder& b) {
        if (a.recs.size() != b.recs.size()) return false;
        for (size_t k = 0; k < a.recs.size(); ++k) {
            const LaunchRec &x = a.recs[k], &y = b.recs[k];
            if (x.fn != y.fn || x.grid.x != y.grid.x || x.grid.y != y.grid.y || x.grid.z != y.grid.z ||
                x.block.x != y.block.x || x.block.y != y.block.y || x.block.z != y.block.z || x.args.size() != y.args.size())
                return false;
        }
        return true;
    };
    std::vector<std::vector<int>> groups;
    for (int i = 0; i < n; ++i) {
        size_t g = 0;
        while (g < groups.size() && !same(recs[groups[g][0]], recs[i])) ++g;
        if (g == groups.size()) groups.emplace_back();
        groups[g].push_back(i);
    }
    // a batched launch multiplies one grid dimension by the group size (x, whose threads must stay
    // below 2^32, or y or z, at most 65535): groups larger than every launch allows are split
    {
        std::vector<std::vector<int>> split;
        for (const std::vector<int>& gr : groups) {
            long long cap = 4096;
            for (const LaunchRec& r : recs[gr[0]].recs) {
                cap = std::min(cap, 65535LL / std::max(r.grid.y, r.grid.z));
                cap = std::min(cap, 0xffffffffLL / ((long long)r.grid.x * r.block.x * r.block.y * r.block.z));
            }
            cap = std::max(cap, 1LL);
            for (size_t a = 0; a < gr.size(); a += (size_t)cap)
                split.emplace_back(gr.begin() + a, gr.begin() + std::min(gr.size(), a + (size_t)cap));
        }
        groups.swap(split);
    }
    // argument tables: for every group and position, the members' argument structs back to back
    std::vector<std::vector<size_t>> off(groups.size());
    size_t total = 0;
    for (size_t g = 0; g < groups.size(); ++g)
        for (const LaunchRec& r : recs[groups[g][0]].recs) {
            off[g].push_back(total);
            total += (r.args.size() * groups[g].size() + 255) / 256 * 256;
        }
    std::vector<unsigned char> host(std::max<size_t>(total, 256));
    for (size_t g = 0; g < groups.size(); ++g)
        for (size_t k = 0; k < off[g].size(); ++k)
            for (size_t m = 0; m < groups[g].size(); ++m) {
                const LaunchRec& r = recs[groups[g][m]].recs[k];
                std::memcpy(host.data() + off[g][k] + m * r.args.size(), r.args.data(), r.args.size());
            }
    auto graph_holder = std::make_unique<BatchGraph>();
    NSLGF_TRY(graph_holder->desc.ensure(host.size()));
    NSLGF_HIP_CHECK(hipMemcpy(graph_holder->desc.p, host.data(), host.size(), hipMemcpyHostToDevice));
    const int nb = std::min((int)groups.size(), 16);
    while ((int)h->branches.size() < nb) {
        hipStream_t bs;
        NSLGF_HIP_CHECK(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
        h->branches.push_back(bs);
    }
    while ((int)h->batch_events.size() < nb + 1) {
        hipEvent_t e;
        NSLGF_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        h->batch_events.push_back(e);
    }
    if (!h->capture) NSLGF_HIP_CHECK(hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    int rc = NSLGF_OK, launches = 0;
    if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeRelaxed) != hipSuccess) {
        set_error("herk_step_batched: stream capture could not start");
        rc = NSLGF_EHIP;
    }
    if (rc == NSLGF_OK && hipEventRecord(h->batch_events[0], h->capture) != hipSuccess) rc = NSLGF_EHIP;
    for (int b = 0; rc == NSLGF_OK && b < nb; ++b)
        if (hipStreamWaitEvent(h->branches[b], h->batch_events[0], 0) != hipSuccess) rc = NSLGF_EHIP;
    for (size_t g = 0; rc == NSLGF_OK && g < groups.size(); ++g) {
        const std::vector<LaunchRec>& rs = recs[groups[g][0]].recs;
        for (size_t k = 0; rc == NSLGF_OK && k < rs.size(); ++k, ++launches)
            rc = rs[k].fn((const char*)graph_holder->desc.p + off[g][k], (int)groups[g].size(), rs[k].grid,
                          rs[k].block, h->branches[g % nb]);
    }
    for (int b = 0; rc == NSLGF_OK && b < nb; ++b) {
        if (hipEventRecord(h->batch_events[b + 1], h->branches[b]) != hipSuccess ||
            hipStreamWaitEvent(h->capture, h->batch_events[b + 1], 0) != hipSuccess)
            rc = NSLGF_EHIP;
    }
    const hipError_t ec = hipStreamEndCapture(h->capture, &graph);
    if (rc == NSLGF_OK && ec != hipSuccess) {
        set_error(std::string("herk_step_batched: capture failed: ") + hipGetErrorString(ec));
        rc = NSLGF_EHIP;
    }
    if (rc == NSLGF_OK && hipGraphInstantiate(&graph_holder->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
        set_error("herk_step_batched: graph instantiation failed");
        rc = NSLGF_EHIP;
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (rc != NSLGF_OK) {
        (void)hipGetLastError();
        return rc;
    }
    graph_holder->key = key;
    graph_holder->groups = (int)groups.size();
    graph_holder->launches = launches;
    h->batch = std::move(graph_holder);
    return NSLGF_OK;
}

// Reads a guarded step's accumulators back (synchronising the stream): st->div_max, and
// NSLGF_ENONFINITE if a non-finite value was seen.
static int read_guard(nslgf_state* st, const unsigned long long* acc, hipStream_t s) {
    unsigned long long host[2];
    NSLGF_HIP_CHECK(hipMemcpyAsync(host, acc, sizeof host, hipMemcpyDeviceToHost, s));
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    std::memcpy(&st->div_max, &host[0], sizeof(double));
    if (host[1]) {
        set_error("herk_step: " + std::to_string(host[1]) + " non-finite values in the step's velocity or pressure");
        return NSLGF_ENONFINITE;
    }
    return NSLGF_OK;
}

}  // namespace nslgf

using namespace nslgf;

#define NSLGF_ENTER(h)                                                                             \
    do {                                                                                           \
        if (!(h)) {                                                                                \
            set_error("null handle");                                                              \
            return NSLGF_EINVAL;                                                                   \
        }                                                                                          \
        NSLGF_HIP_CHECK(hipSetDevice((h)->device));                                                \
    } while (0)

namespace nslgf {
int enter_handle(nslgf_t h) {
    NSLGF_ENTER(h);
    return NSLGF_OK;
}
}  // namespace nslgf

extern "C" {

const char* nslgf_last_error(void) { return g_last_error.c_str(); }
const char* nslgf_version(void) { return "nslgf-mi355x 0.1"; }

int nslgf_create(nslgf_t* h, int device) {
    NSLGF_CHECK_ARG(h != nullptr, "nslgf_create: null output pointer");
    int count = 0;
    NSLGF_HIP_CHECK(hipGetDeviceCount(&count));
    NSLGF_CHECK_ARG(device >= 0 && device < count, "nslgf_create: no such device");
    NSLGF_HIP_CHECK(hipSetDevice(device));
    auto* c = new (std::nothrow) nslgf_ctx();
    if (!c) {
        set_error("out of host memory");
        return NSLGF_ENOMEM;
    }
    c->device = device;
    const int rc = scratch_address(device, &c->scratch);
    if (rc != NSLGF_OK) {
        delete c;
        return rc;
    }
    *h = c;
    return NSLGF_OK;
}

int nslgf_destroy(nslgf_t h) {
    if (!h) return NSLGF_OK;
    (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();
    delete h;
    return NSLGF_OK;
}

int lgf_value(int n1, int n2, int n3, double* out) {
    NSLGF_CHECK_ARG(out != nullptr, "lgf_value: null output");
    NSLGF_CHECK_ARG(std::abs(n1) <= 100000 && std::abs(n2) <= 100000 && std::abs(n3) <= 100000, "lgf_value: |n| too large");
    *out = lgf_value_host(n1, n2, n3);
    return NSLGF_OK;
}

int lgf_table(nslgf_t h, int nx, int ny, int nz, int dtype, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    auto key = std::make_tuple(nx, ny, nz, dtype, h->fft_plan);
    if (h->plans.erase(key)) h->batch.reset();  // a captured batch graph holds the erased plan's buffers
    ConvPlan* p = nullptr;
    NSLGF_TRY(build_plan(h, nx, ny, nz, dtype, (hipStream_t)stream, &p));
    // the dtype's twiddle tables too, so that every buffer a convolution of this box reads exists
    const void *a, *b, *c, *d;
    return plan_twiddles(h, *p, dtype, &a, &b, &c, &d);
}

int lgf_convolve(nslgf_t h, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double dx, int dtype,
                 void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(src && dst, "lgf_convolve: null pointer");
    NSLGF_CHECK_ARG(src != dst, "lgf_convolve: src and dst must differ");
    NSLGF_CHECK_ARG(ncomp >= 1 && ncomp <= 3, "lgf_convolve: ncomp must be 1..3");
    NSLGF_CHECK_ARG(std::isfinite(dx) && dx > 0, "lgf_convolve: dx must be > 0");
    ConvPlan* p = nullptr;
    NSLGF_TRY(build_plan(h, nx, ny, nz, dtype, (hipStream_t)stream, &p));
    return run_conv_shared(h, *p, src, dst, ncomp, dx * dx, (hipStream_t)stream);
}

int lgf_convolve_noalloc(nslgf_t h, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double dx,
                         int dtype, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(src && dst, "lgf_convolve_noalloc: null pointer");
    NSLGF_CHECK_ARG(src != dst, "lgf_convolve_noalloc: src and dst must differ");
    NSLGF_CHECK_ARG(ncomp >= 1 && ncomp <= 3, "lgf_convolve_noalloc: ncomp must be 1..3");
    NSLGF_CHECK_ARG(std::isfinite(dx) && dx > 0, "lgf_convolve_noalloc: dx must be > 0");
    auto it = h->plans.find(std::make_tuple(nx, ny, nz, dtype, h->fft_plan));
    if (it == h->plans.end()) {
        set_error("lgf_convolve_noalloc: no plan for this box and dtype; call lgf_table first");
        return NSLGF_ESTATE;
    }
    ConvPlan& p = *it->second;
    const size_t es = dtype_size(dtype);
    const size_t a1 = (size_t)ncomp * conv_ws_elems_a1(p) * es;
    const size_t a1r = (a1 + 255) / 256 * 256;
    const size_t a2 = (size_t)ncomp * conv_ws_elems_a2(p) * es;
    if (a1r + a2 > (size_t)NSLGF_NOALLOC_SCRATCH_BYTES) {
        set_error("lgf_convolve_noalloc: the convolution needs " + std::to_string(a1r + a2) +
                  " bytes of workspace, more than the scratch array's " +
                  std::to_string((size_t)NSLGF_NOALLOC_SCRATCH_BYTES));
        return NSLGF_EINVAL;
    }
    char* base = (char*)h->scratch;  // this device's address of `scratch`, taken when the handle was created
    const bool prof = h->prof.on;     // profiling would create events
    h->prof.on = false;
    h->no_alloc = true;
    const int rc = run_conv(h, p, src, dst, ncomp, dx * dx, (hipStream_t)stream, base, base + a1r);
    h->no_alloc = false;
    h->prof.on = prof;
    return rc;
}

int if_apply(nslgf_t h, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double alpha, int dtype,
             void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(src && dst, "if_apply: null pointer");
    NSLGF_CHECK_ARG(ncomp >= 1 && ncomp <= 6, "if_apply: ncomp must be 1..6");
    NSLGF_CHECK_ARG(std::isfinite(alpha) && alpha >= 0.0, "if_apply: alpha must be >= 0");
    Tuning tn;
    NSLGF_TRY(get_tuning(h, nx, ny, nz, dtype, (hipStream_t)stream, &tn));
    return run_if_shared(h, src, dst, ncomp, nx, ny, nz, alpha, dtype, (hipStream_t)stream, tn);
}

size_t nslgf_state_bytes(int nx, int ny, int nz, int dtype) {
    if (nx < 1 || ny < 1 || nz < 1 || nx > 256 || ny > 256 || nz > 256) return 0;
    return state_guard_offset(nx, ny, nz, dtype) + kGuardBytes;
}

int herk_stage(nslgf_t h, nslgf_state* st, int stage, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(st != nullptr, "herk_stage: null state");
    NSLGF_TRY(check_box(st->nx, st->ny, st->nz));
    NSLGF_TRY(check_dtype(st->dtype));
    NSLGF_CHECK_ARG(st->u && st->d && st->work, "herk_stage: null u, d or work");
    NSLGF_CHECK_ARG(st->scheme >= NSLGF_SCHEME_A && st->scheme <= NSLGF_SCHEME_C, "herk_stage: unknown scheme");
    NSLGF_CHECK_ARG(std::isfinite(st->dt) && st->dt > 0 && std::isfinite(st->dx) && st->dx > 0 &&
                        std::isfinite(st->re) && st->re > 0,
                    "herk_stage: dt, dx and re must be > 0");
    NSLGF_CHECK_ARG(st->n_buf >= 0, "herk_stage: n_buf must be >= 0");
    NSLGF_CHECK_ARG(!(st->supp_blocks || st->soln_blocks) || (st->block >= 1 && st->block <= 256),
                    "herk_stage: block masks need a block size of 1..256 cells");
    if (stage == 1) st->stage_done = 0;
    if (stage != st->stage_done + 1 || stage < 1 || stage > 3) {
        set_error("herk_stage: stages must be called in order 1, 2, 3");
        return NSLGF_ESTATE;
    }
    hipStream_t s = (hipStream_t)stream;
    const int nx = st->nx, ny = st->ny, nz = st->nz, dt_ = st->dtype;
    const long long M = (long long)nx * ny * nz;
    const size_t es = dtype_size(dt_);
    char* w = (char*)st->work;
    const StateLayout L = state_layout(nx, ny, nz);
    void* q = w + L.q * es;
    void* w1 = w + L.w1 * es;
    void* w2 = w + L.w2 * es;
    void* r = w + L.r * es;
    void* dhat = w + L.dhat * es;
    void* t1 = w + L.t1 * es;
    void* t2 = w + L.t2 * es;
    void* a1 = w + L.a1 * es;
    void* a2 = w + L.a2 * es;
    double at[4][4], ct[4];
    tableau(st->scheme, at, ct);
    const double dt = st->dt, beta = dt / (st->dx * st->dx * st->re);
    const double alpha = (ct[stage] - ct[stage - 1]) * beta;
    ConvPlan* plan = nullptr;
    NSLGF_TRY(build_plan(h, nx, ny, nz, dt_, s, &plan));
    Tuning tn;
    NSLGF_TRY(get_tuning(h, nx, ny, nz, dt_, s, &tn));
    StageCoef c{};
    c.nbuf = st->n_buf;
    c.soln_blocks = st->soln_blocks;
    c.nb = st->block;
    c.c_g = -at[stage][stage] * dt;
    const double inv = 1.0 / (at[stage][stage] * dt);
    if (stage == 1) {
        c.c_q = 1.0;
        c.copy_q = 1;
        NSLGF_PROF(h, "stage_rhs", s,
                   launch_stage_rhs(dt_, st->u, q, nullptr, nullptr, r, c, nx, ny, nz, st->dx, s, tn.cell_shape));
    } else if (stage == 2) {
        const double a_prev = (ct[1] - ct[0]) * beta;
        NSLGF_TRY(run_if(h, q, q, 6, nx, ny, nz, a_prev, dt_, s, t1, t2, tn));  // q and w1 are adjacent
        c.c_q = 1.0;
        c.c_w1 = dt * at[2][1];
        NSLGF_PROF(h, "stage_rhs", s,
                   launch_stage_rhs(dt_, st->u, q, w1, nullptr, r, c, nx, ny, nz, st->dx, s, tn.cell_shape));
    } else {
        // final-stage form: r^3 = H^2 (q^2 + dt (a~31 w^{2,1} + a~32 w^{2,2})) + g^3
        const double a_prev = (ct[2] - ct[1]) * beta;
        const IfCombine cb{{q, w1, w2}, {1.0, dt * at[3][1], dt * at[3][2]}};
        NSLGF_TRY(run_if_combined(h, cb, r, 3, nx, ny, nz, a_prev, dt_, s, t1, t2, tn));
        c.c_q = 1.0;
        NSLGF_PROF(h, "stage_rhs", s,
                   launch_stage_rhs(dt_, st->u, r, nullptr, nullptr, r, c, nx, ny, nz, st->dx, s, tn.cell_shape));
    }
    // pressure source M_supp Dbar r, formed while the convolution's first pass loads
    const DivSource dsrc{r, st->n_buf, 1.0 / st->dx, st->supp_blocks, st->block};
    NSLGF_TRY(run_conv(h, *plan, nullptr, dhat, 1, st->dx * st->dx, s, a1, a2, &dsrc));
    // u^i = H^i (r^i - G dhat^i) and w^{i,i} = (g^i - G dhat^i) / (a~_ii dt) = (r^i - G dhat^i - q^i -
    // dt sum_j a~_ij w^{i,j}) / (a~_ii dt); the projection is applied while the IF loads (with H^i = I,
    // e.g. the last stage of Schemes A and B, it writes u directly)
    IfProject pj{dhat, 1.0 / st->dx, nullptr, nullptr, 0.0, 0.0, nullptr, 0.0};
    if (stage == 1) {
        pj.q = q;
        pj.c_q = 1.0;
        pj.wnew = w1;
        pj.inv = inv;
    } else if (stage == 2) {
        pj.q = q;
        pj.w1 = w1;
        pj.c_q = 1.0;
        pj.c_w1 = dt * at[2][1];
        pj.wnew = w2;
        pj.inv = inv;
    }
    NSLGF_TRY(run_if_projected(h, r, pj, st->u, nx, ny, nz, alpha, dt_, st->dx, s, t1, t2, tn));
    if (stage == 3) {
        NSLGF_PROF(h, "axpby", s, launch_axpby(dt_, st->d, dhat, 1.0 / (at[3][3] * dt), nullptr, 0.0, nullptr, 0.0, M, s));
        st->t += dt;
    }
    st->stage_done = stage;
    if (st->guard) {
        // FP64 divergence of the projected u^i on the support away from the buffer (and, last stage, the
        // non-finite test of d too)
        unsigned long long* acc = (unsigned long long*)(w + state_guard_offset(nx, ny, nz, dt_));
        if (stage == 1) NSLGF_TRY(launch_guard_reset(acc, s));
        double wts[kIfMaxRadius + 1];
        const int rad = alpha > 0.0 ? if_weights(alpha, dt_, wts, kIfMaxRadius) : 0;
        const int margin = st->guard_margin > 0 ? st->guard_margin : st->n_buf + std::max(rad, 0) + 1;
        NSLGF_PROF(h, "guard", s, launch_guard(dt_, st->u, stage == 3 ? st->d : nullptr, nx, ny, nz, margin, st->dx,
                                               acc, s));
        if (stage == 3 && !h->capturing) NSLGF_TRY(read_guard(st, acc, s));
    }
    return NSLGF_OK;
}

int herk_check(nslgf_t h, const nslgf_state* st, int margin, double* div_max, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(st != nullptr && div_max != nullptr, "herk_check: null state or output");
    NSLGF_TRY(check_box(st->nx, st->ny, st->nz));
    NSLGF_TRY(check_dtype(st->dtype));
    NSLGF_CHECK_ARG(st->u && st->d, "herk_check: null u or d");
    NSLGF_CHECK_ARG(std::isfinite(st->dx) && st->dx > 0, "herk_check: dx must be > 0");
    NSLGF_CHECK_ARG(margin >= 0, "herk_check: margin must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    NSLGF_TRY(h->partial.ensure(2 * sizeof(unsigned long long)));
    unsigned long long* acc = (unsigned long long*)h->partial.p;
    NSLGF_TRY(launch_guard_reset(acc, s));
    NSLGF_PROF(h, "guard", s, launch_guard(st->dtype, st->u, st->d, st->nx, st->ny, st->nz, margin, st->dx, acc, s));
    unsigned long long host[2];
    NSLGF_HIP_CHECK(hipMemcpyAsync(host, acc, sizeof host, hipMemcpyDeviceToHost, s));
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    std::memcpy(div_max, &host[0], sizeof(double));
    if (host[1]) {
        set_error("herk_check: " + std::to_string(host[1]) + " non-finite values in u or d");
        return NSLGF_ENONFINITE;
    }
    return NSLGF_OK;
}

int herk_step(nslgf_t h, nslgf_state* st, void* stream) {
    for (int i = 1; i <= 3; ++i) NSLGF_TRY(herk_stage(h, st, i, stream));
    return NSLGF_OK;
}

int herk_step_batched(nslgf_t h, nslgf_state* const* sts, int n, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(sts != nullptr && n >= 1 && n <= 4096, "herk_step_batched: need 1..4096 states");
    hipStream_t s = (hipStream_t)stream;
    std::vector<unsigned long long> key;
    key.reserve((size_t)n * 22);
    auto bits = [](double v) {
        unsigned long long b;
        std::memcpy(&b, &v, sizeof b);
        return b;
    };
    for (int i = 0; i < n; ++i) {
        const nslgf_state* st = sts[i];
        NSLGF_CHECK_ARG(st != nullptr, "herk_step_batched: null state");
        NSLGF_TRY(check_box(st->nx, st->ny, st->nz));
        NSLGF_TRY(check_dtype(st->dtype));
        NSLGF_CHECK_ARG(st->u && st->d && st->work, "herk_step_batched: null u, d or work");
        for (int j = 0; j < i; ++j)
            NSLGF_CHECK_ARG(sts[j]->work != st->work && sts[j]->u != st->u,
                            "herk_step_batched: states must not share u or work");
        // plans and twiddles exist before any capture
        ConvPlan* p = nullptr;
        NSLGF_TRY(build_plan(h, st->nx, st->ny, st->nz, st->dtype, s, &p));
        const void *a, *b, *c, *d;
        NSLGF_TRY(plan_twiddles(h, *p, st->dtype, &a, &b, &c, &d));
        Tuning tn;  // (tuned now if the handle tunes, so that the capture only looks it up)
        NSLGF_TRY(get_tuning(h, st->nx, st->ny, st->nz, st->dtype, s, &tn));
        const unsigned long long k[] = {(unsigned long long)tn.if_rows, (unsigned long long)tn.if_seg,
                                        (unsigned long long)tn.cell_shape,(unsigned long long)st->nx, (unsigned long long)st->ny,
                                        (unsigned long long)st->nz, (unsigned long long)st->dtype,
                                        (unsigned long long)st->scheme, (unsigned long long)st->n_buf,
                                        bits(st->dx), bits(st->dt), bits(st->re),
                                        (unsigned long long)(uintptr_t)st->u, (unsigned long long)(uintptr_t)st->d,
                                        (unsigned long long)(uintptr_t)st->work, (unsigned long long)(uintptr_t)p,
                                        (unsigned long long)(uintptr_t)p->khat.p,
                                        (unsigned long long)(uintptr_t)st->supp_blocks,
                                        (unsigned long long)(uintptr_t)st->soln_blocks, (unsigned long long)st->block,
                                        (unsigned long long)st->guard, (unsigned long long)st->guard_margin};
        key.insert(key.end(), std::begin(k), std::end(k));
    }
    if (!h->batch || h->batch->key != key) {
        h->batch.reset();
        if (h->batch_mode == NSLGF_BATCH_PASSES) {
            const int rc = capture_batched_passes(h, sts, n, s, key);
            if (rc != NSLGF_ESTATE) {  // (NSLGF_ESTATE: a step has no batched form; capture it per problem)
                NSLGF_TRY(rc);
            }
        }
    }
    if (!h->batch || h->batch->key != key) {
        h->batch.reset();
        const int nb = std::min(n, 16);
        while ((int)h->branches.size() < nb) {
            hipStream_t bs;
            NSLGF_HIP_CHECK(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
            h->branches.push_back(bs);
        }
        while ((int)h->batch_events.size() < nb + 1) {
            hipEvent_t e;
            NSLGF_HIP_CHECK(hipEventCreateWithFlags(&e, hipEventDisableTiming));
            h->batch_events.push_back(e);
        }
        if (!h->capture) NSLGF_HIP_CHECK(hipStreamCreateWithFlags(&h->capture, hipStreamNonBlocking));
        const bool prof_was = h->prof.on;
        h->prof.on = false;
        std::vector<nslgf_state> saved(n);
        for (int i = 0; i < n; ++i) saved[i] = *sts[i];
        hipGraph_t graph = nullptr;
        int rc = NSLGF_OK;
        if (hipStreamBeginCapture(h->capture, hipStreamCaptureModeRelaxed) != hipSuccess) {
            set_error("herk_step_batched: stream capture could not start");
            rc = NSLGF_EHIP;
        }
        if (rc == NSLGF_OK && hipEventRecord(h->batch_events[0], h->capture) != hipSuccess) rc = NSLGF_EHIP;
        for (int b = 0; rc == NSLGF_OK && b < nb; ++b)
            if (hipStreamWaitEvent(h->branches[b], h->batch_events[0], 0) != hipSuccess) rc = NSLGF_EHIP;
        h->capturing = true;
        for (int i = 0; rc == NSLGF_OK && i < n; ++i) rc = herk_step(h, sts[i], h->branches[i % nb]);
        h->capturing = false;
        for (int b = 0; rc == NSLGF_OK && b < nb; ++b) {
            if (hipEventRecord(h->batch_events[b + 1], h->branches[b]) != hipSuccess ||
                hipStreamWaitEvent(h->capture, h->batch_events[b + 1], 0) != hipSuccess)
                rc = NSLGF_EHIP;
        }
        const hipError_t ec = hipStreamEndCapture(h->capture, &graph);
        if (rc == NSLGF_OK && ec != hipSuccess) {
            set_error(std::string("herk_step_batched: capture failed: ") + hipGetErrorString(ec));
            rc = NSLGF_EHIP;
        }
        for (int i = 0; i < n; ++i) *sts[i] = saved[i];
        h->prof.on = prof_was;
        auto g = std::make_unique<BatchGraph>();
        if (rc == NSLGF_OK && hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0) != hipSuccess) {
            set_error("herk_step_batched: graph instantiation failed");
            rc = NSLGF_EHIP;
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (rc != NSLGF_OK) {
            (void)hipGetLastError();
            return rc;
        }
        g->key = key;
        h->batch = std::move(g);
    }
    {
        ProfScope ps(h, "batch_graph", s);
        NSLGF_HIP_CHECK(hipGraphLaunch(h->batch->exec, s));
    }
    int rc = NSLGF_OK;
    for (int i = 0; i < n; ++i) {
        sts[i]->t += sts[i]->dt;
        sts[i]->stage_done = 3;
        if (sts[i]->guard) {
            const unsigned long long* acc = (const unsigned long long*)((const char*)sts[i]->work +
                                                                        state_guard_offset(sts[i]->nx, sts[i]->ny,
                                                                                           sts[i]->nz, sts[i]->dtype));
            const int g = read_guard(sts[i], acc, s);
            if (rc == NSLGF_OK) rc = g;
        }
    }
    return rc;
}

int vor2vel(nslgf_t h, const void* w, void* u, int nx, int ny, int nz, double dx, int dtype, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(w && u && w != u, "vor2vel: null or aliased pointers");
    NSLGF_CHECK_ARG(std::isfinite(dx) && dx > 0, "vor2vel: dx must be > 0");
    hipStream_t s = (hipStream_t)stream;
    ConvPlan* p = nullptr;
    NSLGF_TRY(build_plan(h, nx, ny, nz, dtype, s, &p));
    const long long M = (long long)nx * ny * nz;
    NSLGF_TRY(h->tmp3.ensure((size_t)3 * M * dtype_size(dtype)));
    Tuning tn;
    NSLGF_TRY(get_tuning(h, nx, ny, nz, dtype, s, &tn));
    NSLGF_TRY(run_conv_shared(h, *p, w, h->tmp3.p, 3, -dx * dx, s));  // a = -L^{-1} w
    NSLGF_PROF(h, "curl_bar", s,
               launch_stencil(NSLGF_OP_CURL_BAR, dtype, h->tmp3.p, u, 3, nx, ny, nz, dx, s, tn.cell_shape));
    return NSLGF_OK;
}

// u = Cbar a, a = -L^{-1} w, w = M_supp C u, through two 3-component temporaries.
static int refresh_into(nslgf_t h, void* u, int nx, int ny, int nz, int n_buf, double dx, int dtype, void* wbuf,
                        void* abuf, hipStream_t s, const unsigned char* blocks = nullptr, int nb = 0) {
    ConvPlan* p = nullptr;
    NSLGF_TRY(build_plan(h, nx, ny, nz, dtype, s, &p));
    Tuning tn;
    NSLGF_TRY(get_tuning(h, nx, ny, nz, dtype, s, &tn));
    NSLGF_PROF(h, "curl_masked", s,
               launch_masked_curl(dtype, u, wbuf, n_buf, blocks, nb, nx, ny, nz, dx, s, tn.cell_shape));
    NSLGF_TRY(run_conv_shared(h, *p, wbuf, abuf, 3, -dx * dx, s));
    NSLGF_PROF(h, "curl_bar", s, launch_stencil(NSLGF_OP_CURL_BAR, dtype, abuf, u, 3, nx, ny, nz, dx, s, tn.cell_shape));
    return NSLGF_OK;
}

static int max_abs_host(nslgf_t h, const void* u, int nx, int ny, int nz, int n_buf, int dtype, double* out,
                        hipStream_t s) {
    const int nb = 1024;
    NSLGF_TRY(h->partial.ensure(nb * sizeof(double)));
    NSLGF_TRY(launch_max_abs(dtype, u, n_buf, nx, ny, nz, (double*)h->partial.p, nb, s));
    std::vector<double> host(nb);
    NSLGF_HIP_CHECK(hipMemcpyAsync(host.data(), h->partial.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    double m = 0.0;
    for (double v : host) m = v > m ? v : m;
    *out = m;
    return NSLGF_OK;
}

int if_trunc_error(double alpha, int k, double* out) {
    NSLGF_CHECK_ARG(out != nullptr, "if_trunc_error: null output");
    NSLGF_CHECK_ARG(std::isfinite(alpha) && alpha >= 0.0, "if_trunc_error: alpha must be a finite value >= 0");
    NSLGF_CHECK_ARG(k >= 1, "if_trunc_error: k must be >= 1");
    *out = if_trunc_error_host(alpha, k);
    return NSLGF_OK;
}

int refresh_interval(double beta, int n_buf, double umax, double eps, int q_cap, int* q_max) {
    NSLGF_CHECK_ARG(q_max != nullptr, "refresh_interval: null output");
    NSLGF_CHECK_ARG(std::isfinite(beta) && beta >= 0.0, "refresh_interval: beta must be a finite value >= 0");
    NSLGF_CHECK_ARG(n_buf >= 0, "refresh_interval: n_buf must be >= 0");
    NSLGF_CHECK_ARG(std::isfinite(umax) && umax >= 0.0, "refresh_interval: umax must be a finite value >= 0");
    NSLGF_CHECK_ARG(std::isfinite(eps) && eps > 0.0, "refresh_interval: eps must be > 0");
    NSLGF_CHECK_ARG(q_cap >= 1, "refresh_interval: q_cap must be >= 1");
    *q_max = refresh_interval_host(beta, n_buf, umax, eps, q_cap);
    return NSLGF_OK;
}

int max_component_abs(nslgf_t h, const void* u, int nx, int ny, int nz, int n_buf, int dtype, double* out,
                      void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(u && out, "max_component_abs: null pointer");
    NSLGF_CHECK_ARG(n_buf >= 0, "max_component_abs: n_buf must be >= 0");
    return max_abs_host(h, u, nx, ny, nz, n_buf, dtype, out, (hipStream_t)stream);
}

int velocity_refresh(nslgf_t h, void* u, int nx, int ny, int nz, int n_buf, double dx, int dtype, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(u != nullptr, "velocity_refresh: null pointer");
    NSLGF_CHECK_ARG(n_buf >= 0, "velocity_refresh: n_buf must be >= 0");
    NSLGF_CHECK_ARG(std::isfinite(dx) && dx > 0, "velocity_refresh: dx must be > 0");
    const size_t bytes = (size_t)3 * nx * ny * nz * dtype_size(dtype);
    NSLGF_TRY(h->tmp3.ensure(bytes));
    NSLGF_TRY(h->tmp3b.ensure(bytes));
    return refresh_into(h, u, nx, ny, nz, n_buf, dx, dtype, h->tmp3b.p, h->tmp3.p, (hipStream_t)stream);
}

int herk_run(nslgf_t h, nslgf_state* st, int nsteps, double eps, int q_cap, int* refreshes, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(st != nullptr, "herk_run: null state");
    NSLGF_TRY(check_box(st->nx, st->ny, st->nz));
    NSLGF_TRY(check_dtype(st->dtype));
    NSLGF_CHECK_ARG(st->u && st->d && st->work, "herk_run: null u, d or work");
    NSLGF_CHECK_ARG(nsteps >= 0, "herk_run: nsteps must be >= 0");
    NSLGF_CHECK_ARG(std::isfinite(eps) && eps > 0.0, "herk_run: eps must be > 0");
    NSLGF_CHECK_ARG(q_cap >= 1, "herk_run: q_cap must be >= 1");
    NSLGF_CHECK_ARG(std::isfinite(st->dt) && st->dt > 0 && std::isfinite(st->dx) && st->dx > 0 &&
                        std::isfinite(st->re) && st->re > 0 && st->n_buf >= 0,
                    "herk_run: dt, dx and re must be > 0 and n_buf >= 0");
    hipStream_t s = (hipStream_t)stream;
    const int nx = st->nx, ny = st->ny, nz = st->nz, dt_ = st->dtype;
    const double beta = st->dt / (st->dx * st->dx * st->re);
    // the refresh works in the state's IF temporaries (6 components), which no stage keeps
    const StateLayout L = state_layout(nx, ny, nz);
    const size_t es = dtype_size(dt_);
    char* wbase = (char*)st->work + L.t1 * es;
    char* abase = wbase + (size_t)3 * nx * ny * nz * es;
    auto interval = [&](int* q) -> int {
        double umax = 0.0;
        NSLGF_TRY(max_abs_host(h, st->u, nx, ny, nz, st->n_buf, dt_, &umax, s));
        *q = refresh_interval_host(beta, st->n_buf, umax, eps, q_cap);
        if (*q == 0) {
            set_error("herk_run: the buffer is too thin for eps (one step already exceeds it)");
            return NSLGF_EINVAL;
        }
        return NSLGF_OK;
    };
    int q_max = 0, count = 0, nref = 0;
    NSLGF_TRY(interval(&q_max));
    for (int n = 0; n < nsteps; ++n) {
        NSLGF_TRY(herk_step(h, st, stream));
        if (++count == q_max) {
            NSLGF_TRY(refresh_into(h, st->u, nx, ny, nz, st->n_buf, st->dx, dt_, wbase, abase, s));
            ++nref;
            count = 0;
            NSLGF_TRY(interval(&q_max));
        }
    }
    if (refreshes) *refreshes = nref;
    return NSLGF_OK;
}

int flow_diagnostics(nslgf_t h, const void* u, int nx, int ny, int nz, int n_buf, double dx, const double* origin,
                     int dtype, double* out, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(u && origin && out, "flow_diagnostics: null pointer");
    NSLGF_CHECK_ARG(std::isfinite(dx) && dx > 0, "flow_diagnostics: dx must be > 0");
    NSLGF_CHECK_ARG(n_buf >= 0, "flow_diagnostics: n_buf must be >= 0");
    NSLGF_CHECK_ARG(std::isfinite(origin[0]) && std::isfinite(origin[1]) && std::isfinite(origin[2]),
                    "flow_diagnostics: origin must be finite");
    const int nb = 1024;
    NSLGF_TRY(h->partial.ensure((size_t)nb * kDiagnosticSums * sizeof(double)));
    hipStream_t s = (hipStream_t)stream;
    NSLGF_PROF(h, "diagnostics", s, launch_diagnostics(dtype, u, n_buf, nx, ny, nz, dx, origin, (double*)h->partial.p, nb, s));
    std::vector<double> host((size_t)nb * kDiagnosticSums);
    NSLGF_HIP_CHECK(hipMemcpyAsync(host.data(), h->partial.p, host.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    double sum[kDiagnosticSums] = {};
    for (int b = 0; b < nb; ++b)  // fixed order: the result does not depend on scheduling
        for (int v = 0; v < kDiagnosticSums; ++v) sum[v] += host[(size_t)b * kDiagnosticSums + v];
    const double dv = dx * dx * dx;
    double I[3];
    for (int q = 0; q < 3; ++q) I[q] = 0.5 * dv * sum[q];
    const double I2 = I[0] * I[0] + I[1] * I[1] + I[2] * I[2];
    for (int q = 0; q < 3; ++q) out[q] = I[q];
    out[3] = dv * sum[13];        // K
    out[4] = 0.5 * dv * sum[12];  // E
    out[5] = dv * sum[14];        // J
    for (int p = 0; p < 3; ++p) {  // X (undefined without impulse: NaN)
        double m = 0.0;
        for (int q = 0; q < 3; ++q) m += I[q] * sum[3 + 3 * q + p];
        out[6 + p] = I2 > 0.0 ? 0.5 * dv * m / I2 : std::nan("");
    }
    return NSLGF_OK;
}

int block_weights(nslgf_t h, const void* u, int nx, int ny, int nz, int nb, int n_buf, double dx, int dtype, double* mu,
                  double* nu, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(u && mu && nu, "block_weights: null pointer");
    NSLGF_CHECK_ARG(nb >= 1 && nb <= 256, "block_weights: nb must be 1..256");
    NSLGF_CHECK_ARG(n_buf >= 0, "block_weights: n_buf must be >= 0");
    NSLGF_CHECK_ARG(std::isfinite(dx) && dx > 0, "block_weights: dx must be > 0");
    hipStream_t s = (hipStream_t)stream;
    const long long M = (long long)nx * ny * nz;
    const long long nblocks = (long long)((nx + nb - 1) / nb) * ((ny + nb - 1) / nb) * ((nz + nb - 1) / nb);
    NSLGF_TRY(h->tmp3.ensure((size_t)3 * M * dtype_size(dtype)));
    NSLGF_TRY(h->partial.ensure((size_t)2 * nblocks * sizeof(double)));
    double* dmu = (double*)h->partial.p;
    NSLGF_PROF(h, "nonlinear", s, launch_stencil(NSLGF_OP_NONLINEAR, dtype, u, h->tmp3.p, 3, nx, ny, nz, dx, s));
    NSLGF_PROF(h, "block_weights", s,
               launch_block_weights(dtype, u, h->tmp3.p, nx, ny, nz, nb, n_buf, dx, dmu, dmu + nblocks, s));
    NSLGF_HIP_CHECK(hipMemcpyAsync(mu, dmu, nblocks * sizeof(double), hipMemcpyDeviceToHost, s));
    NSLGF_HIP_CHECK(hipMemcpyAsync(nu, dmu + nblocks, nblocks * sizeof(double), hipMemcpyDeviceToHost, s));
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    return NSLGF_OK;
}

int classify_blocks(const double* mu, const double* nu, int bx, int by, int bz, double eps_supp, double eps_soln,
                    int n_xb, double* W, unsigned char* supp, unsigned char* soln, unsigned char* xsoln) {
    NSLGF_CHECK_ARG(mu && nu && supp && soln && xsoln, "classify_blocks: null pointer");
    NSLGF_CHECK_ARG(bx >= 1 && by >= 1 && bz >= 1, "classify_blocks: the block grid must be non-empty");
    NSLGF_CHECK_ARG(std::isfinite(eps_supp) && std::isfinite(eps_soln) && eps_supp >= 0 && eps_soln >= 0,
                    "classify_blocks: thresholds must be finite and >= 0");
    NSLGF_CHECK_ARG(n_xb >= 0, "classify_blocks: n_xb must be >= 0");
    const long long n = (long long)bx * by * bz;
    for (long long b = 0; b < n; ++b)
        NSLGF_CHECK_ARG(std::isfinite(mu[b]) && std::isfinite(nu[b]) && mu[b] >= 0 && nu[b] >= 0,
                        "classify_blocks: weights must be finite and >= 0");
    classify_blocks_host(mu, nu, bx, by, bz, eps_supp, eps_soln, n_xb, W, supp, soln, xsoln);
    return NSLGF_OK;
}

int herk_run_adaptive(nslgf_t h, nslgf_state* st, int nsteps, int block, double eps_supp, double eps_soln, int n_xb,
                      int* reinits, int* edge_steps, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(st != nullptr, "herk_run_adaptive: null state");
    NSLGF_TRY(check_box(st->nx, st->ny, st->nz));
    NSLGF_TRY(check_dtype(st->dtype));
    NSLGF_CHECK_ARG(st->u && st->d && st->work, "herk_run_adaptive: null u, d or work");
    NSLGF_CHECK_ARG(nsteps >= 0, "herk_run_adaptive: nsteps must be >= 0");
    NSLGF_CHECK_ARG(block >= 1 && block <= 256, "herk_run_adaptive: block must be 1..256");
    NSLGF_CHECK_ARG(std::isfinite(eps_supp) && std::isfinite(eps_soln) && eps_supp >= 0 && eps_soln >= 0,
                    "herk_run_adaptive: thresholds must be finite and >= 0");
    NSLGF_CHECK_ARG(n_xb >= 0, "herk_run_adaptive: n_xb must be >= 0");
    NSLGF_CHECK_ARG(std::isfinite(st->dx) && st->dx > 0 && st->n_buf >= 0,
                    "herk_run_adaptive: dx must be > 0 and n_buf >= 0");
    hipStream_t s = (hipStream_t)stream;
    const int nx = st->nx, ny = st->ny, nz = st->nz, dt_ = st->dtype;
    const int bx = (nx + block - 1) / block, by = (ny + block - 1) / block, bz = (nz + block - 1) / block;
    const long long nbk = (long long)bx * by * bz;
    const long long M = (long long)nx * ny * nz;
    NSLGF_TRY(h->tmp3.ensure((size_t)3 * M * dtype_size(dt_)));
    NSLGF_TRY(h->partial.ensure((size_t)2 * nbk * sizeof(double)));
    NSLGF_TRY(h->blockmask.ensure((size_t)2 * nbk));
    unsigned char* dsupp = (unsigned char*)h->blockmask.p;
    unsigned char* dsoln = dsupp + nbk;
    double* dmu = (double*)h->partial.p;
    std::vector<double> mu(nbk), nu(nbk);
    std::vector<unsigned char> supp(nbk), soln(nbk), xsoln(nbk), psupp, psoln;
    const StateLayout L = state_layout(nx, ny, nz);
    const size_t es = dtype_size(dt_);
    char* wbase = (char*)st->work + L.t1 * es;
    char* abase = wbase + (size_t)3 * M * es;
    int nre = 0, nedge = 0;
    // the state's own domain (its masks or the n_buf rule) is back in place on every return: the
    // masks of this run live in handle memory that the next adaptive run reuses
    struct RestoreMasks {
        nslgf_state* st;
        const unsigned char *supp, *soln;
        int block;
        ~RestoreMasks() {
            st->supp_blocks = supp;
            st->soln_blocks = soln;
            st->block = block;
        }
    } restore{st, st->supp_blocks, st->soln_blocks, st->block};
    for (int step = 0; step < nsteps; ++step) {
        // the domain of this step from the block weights of u (Sec. 4.3)
        NSLGF_PROF(h, "nonlinear", s, launch_stencil(NSLGF_OP_NONLINEAR, dt_, st->u, h->tmp3.p, 3, nx, ny, nz, st->dx, s));
        NSLGF_PROF(h, "block_weights", s,
                   launch_block_weights(dt_, st->u, h->tmp3.p, nx, ny, nz, block, st->n_buf, st->dx, dmu, dmu + nbk, s));
        NSLGF_HIP_CHECK(hipMemcpyAsync(mu.data(), dmu, nbk * sizeof(double), hipMemcpyDeviceToHost, s));
        NSLGF_HIP_CHECK(hipMemcpyAsync(nu.data(), dmu + nbk, nbk * sizeof(double), hipMemcpyDeviceToHost, s));
        NSLGF_HIP_CHECK(hipStreamSynchronize(s));
        classify_blocks_host(mu.data(), nu.data(), bx, by, bz, eps_supp, eps_soln, n_xb, nullptr, supp.data(),
                             soln.data(), xsoln.data());
        bool edge = false;
        for (int k = 0; k < bz && !edge; ++k)
            for (int j = 0; j < by && !edge; ++j)
                for (int i = 0; i < bx && !edge; ++i)
                    if ((i == 0 || j == 0 || k == 0 || i == bx - 1 || j == by - 1 || k == bz - 1) &&
                        xsoln[((long long)k * by + j) * bx + i])
                        edge = true;
        nedge += edge ? 1 : 0;
        const bool first = psupp.empty();
        const bool changed = first || psupp != supp || psoln != soln;
        if (changed) {
            NSLGF_HIP_CHECK(hipMemcpyAsync(dsupp, supp.data(), nbk, hipMemcpyHostToDevice, s));
            NSLGF_HIP_CHECK(hipMemcpyAsync(dsoln, soln.data(), nbk, hipMemcpyHostToDevice, s));
            NSLGF_HIP_CHECK(hipStreamSynchronize(s));  // the host masks are reused below
            psupp = supp;
            psoln = soln;
        }
        if (changed && !first) {
            // re-initialise: u from the vorticity on the new support (Eq. vel_refresh)
            NSLGF_TRY(refresh_into(h, st->u, nx, ny, nz, st->n_buf, st->dx, dt_, wbase, abase, s, dsupp, block));
            ++nre;
        }
        st->supp_blocks = dsupp;
        st->soln_blocks = dsoln;
        st->block = block;
        NSLGF_TRY(herk_step(h, st, stream));
    }
    if (reinits) *reinits = nre;
    if (edge_steps) *edge_steps = nedge;
    return NSLGF_OK;
}

int herk_run_active(nslgf_t h, nslgf_state* st, int nsteps, int block, double eps_supp, double eps_soln, int n_xb,
                    int* reinits, int* regrids, int* box, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(st != nullptr, "herk_run_active: null state");
    NSLGF_TRY(check_box(st->nx, st->ny, st->nz));
    NSLGF_TRY(check_dtype(st->dtype));
    NSLGF_CHECK_ARG(st->u && st->d, "herk_run_active: null u or d");
    NSLGF_CHECK_ARG(nsteps >= 0, "herk_run_active: nsteps must be >= 0");
    NSLGF_CHECK_ARG(block >= 1 && block <= 256, "herk_run_active: block must be 1..256");
    NSLGF_CHECK_ARG(st->nx % block == 0 && st->ny % block == 0 && st->nz % block == 0,
                    "herk_run_active: the grid sizes must be multiples of the block size");
    NSLGF_CHECK_ARG(std::isfinite(eps_supp) && std::isfinite(eps_soln) && eps_supp >= 0 && eps_soln >= 0,
                    "herk_run_active: thresholds must be finite and >= 0");
    NSLGF_CHECK_ARG(n_xb >= 0, "herk_run_active: n_xb must be >= 0");
    NSLGF_CHECK_ARG(std::isfinite(st->dt) && st->dt > 0 && std::isfinite(st->dx) && st->dx > 0 &&
                        std::isfinite(st->re) && st->re > 0 && st->n_buf >= 0,
                    "herk_run_active: dt, dx and re must be > 0 and n_buf >= 0");
    NSLGF_CHECK_ARG(st->scheme >= NSLGF_SCHEME_A && st->scheme <= NSLGF_SCHEME_C, "herk_run_active: unknown scheme");
    hipStream_t s = (hipStream_t)stream;
    const int dt_ = st->dtype;
    const size_t es = dtype_size(dt_);
    // block grid of the whole grid G, (x, y, z) order; the box is [lo, hi) in blocks
    const int gb[3] = {st->nx / block, st->ny / block, st->nz / block};
    const long long gnb = (long long)gb[0] * gb[1] * gb[2];
    int lo[3] = {0, 0, 0}, hi[3] = {gb[0], gb[1], gb[2]};
    auto cells = [&](const int* l, const int* u, int* n) {
        for (int a = 0; a < 3; ++a) n[a] = (u[a] - l[a]) * block;
    };
    int bn[3];
    cells(lo, hi, bn);
    int cur = 0;
    NSLGF_TRY(h->act_u[cur].ensure((size_t)3 * bn[0] * bn[1] * bn[2] * es));
    NSLGF_HIP_CHECK(hipMemcpyAsync(h->act_u[cur].p, st->u, (size_t)3 * bn[0] * bn[1] * bn[2] * es,
                                   hipMemcpyDeviceToDevice, s));
    std::vector<unsigned char> gs(gnb), gn(gnb), gx(gnb), ps, pn;
    int nre = 0, nrg = 0;
    for (int step = 0; step < nsteps; ++step) {
        const long long M = (long long)bn[0] * bn[1] * bn[2];
        const int bb[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
        const long long nbk = (long long)bb[0] * bb[1] * bb[2];
        // classification on the current box (block weights of its velocity, Sec. 4.3)
        NSLGF_TRY(h->tmp3.ensure((size_t)3 * M * es));
        NSLGF_TRY(h->partial.ensure((size_t)2 * nbk * sizeof(double)));
        double* dmu = (double*)h->partial.p;
        void* U = h->act_u[cur].p;
        NSLGF_PROF(h, "nonlinear", s, launch_stencil(NSLGF_OP_NONLINEAR, dt_, U, h->tmp3.p, 3, bn[0], bn[1], bn[2], st->dx, s));
        NSLGF_PROF(h, "block_weights", s, launch_block_weights(dt_, U, h->tmp3.p, bn[0], bn[1], bn[2], block, st->n_buf,
                                                               st->dx, dmu, dmu + nbk, s));
        std::vector<double> mu(nbk), nu(nbk);
        NSLGF_HIP_CHECK(hipMemcpyAsync(mu.data(), dmu, nbk * sizeof(double), hipMemcpyDeviceToHost, s));
        NSLGF_HIP_CHECK(hipMemcpyAsync(nu.data(), dmu + nbk, nbk * sizeof(double), hipMemcpyDeviceToHost, s));
        NSLGF_HIP_CHECK(hipStreamSynchronize(s));
        std::vector<unsigned char> supp(nbk), soln(nbk), xs(nbk);
        classify_blocks_host(mu.data(), nu.data(), bb[0], bb[1], bb[2], eps_supp, eps_soln, 0, nullptr, supp.data(),
                             soln.data(), xs.data());
        // D_supp, D_soln (united with D_supp) in the block coordinates of G, then D_xsoln and its bounding box
        std::fill(gs.begin(), gs.end(), 0);
        std::fill(gn.begin(), gn.end(), 0);
        std::fill(gx.begin(), gx.end(), 0);
        auto gidx = [&](int i, int j, int k) { return ((long long)k * gb[1] + j) * gb[0] + i; };
        for (int k = 0; k < bb[2]; ++k)
            for (int j = 0; j < bb[1]; ++j)
                for (int i = 0; i < bb[0]; ++i) {
                    const long long b = ((long long)k * bb[1] + j) * bb[0] + i;
                    gs[gidx(lo[0] + i, lo[1] + j, lo[2] + k)] = supp[b];
                    gn[gidx(lo[0] + i, lo[1] + j, lo[2] + k)] = (soln[b] || supp[b]) ? 1 : 0;
                }
        int nlo[3] = {gb[0], gb[1], gb[2]}, nhi[3] = {0, 0, 0};
        for (int k = 0; k < gb[2]; ++k)
            for (int j = 0; j < gb[1]; ++j)
                for (int i = 0; i < gb[0]; ++i) {
                    if (!gn[gidx(i, j, k)]) continue;
                    const int c[3] = {i, j, k};
                    for (int a = 0; a < 3; ++a) {
                        nlo[a] = std::min(nlo[a], std::max(0, c[a] - n_xb));
                        nhi[a] = std::max(nhi[a], std::min(gb[a], c[a] + n_xb + 1));
                    }
                }
        if (nhi[0] <= nlo[0]) {  // no solution block at all (a vanishing flow): keep the box
            for (int a = 0; a < 3; ++a) {
                nlo[a] = lo[a];
                nhi[a] = hi[a];
            }
        }
        const bool first = ps.empty();
        const bool changed = !first && (ps != gs || pn != gn);
        const bool moved = nlo[0] != lo[0] || nlo[1] != lo[1] || nlo[2] != lo[2] || nhi[0] != hi[0] ||
                           nhi[1] != hi[1] || nhi[2] != hi[2];
        int nn[3];
        cells(nlo, nhi, nn);
        const long long Mn = (long long)nn[0] * nn[1] * nn[2];
        // the overlap of the old and the new box, in the cell offsets of each
        int soff[3], doff[3], ext[3];
        for (int a = 0; a < 3; ++a) {
            const int l = std::max(lo[a], nlo[a]), u = std::min(hi[a], nhi[a]);
            soff[a] = (l - lo[a]) * block;
            doff[a] = (l - nlo[a]) * block;
            ext[a] = std::max(0, u - l) * block;
        }
        const int nxt = 1 - cur;
        if (first && moved) {
            // the first classification only sets the domain: u restricted to the new box
            NSLGF_TRY(h->act_u[nxt].ensure((size_t)3 * Mn * es));
            NSLGF_TRY(launch_zero(dt_, h->act_u[nxt].p, 3 * Mn, s));
            NSLGF_TRY(launch_copy_box(dt_, U, bn, soff, h->act_u[nxt].p, nn, doff, ext, 3, s));
            cur = nxt;
        } else if (changed) {
            // grid update and re-initialisation: the vorticity on the new support, taken on the old box,
            // moves to the new box, where Vor2Vel gives the velocity (Sec. 5; Eq. vel_refresh)
            std::vector<unsigned char> osupp(nbk);
            for (int k = 0; k < bb[2]; ++k)
                for (int j = 0; j < bb[1]; ++j)
                    for (int i = 0; i < bb[0]; ++i)
                        osupp[((long long)k * bb[1] + j) * bb[0] + i] = gs[gidx(lo[0] + i, lo[1] + j, lo[2] + k)];
            NSLGF_TRY(h->act_mask.ensure((size_t)nbk));
            NSLGF_HIP_CHECK(hipMemcpyAsync(h->act_mask.p, osupp.data(), nbk, hipMemcpyHostToDevice, s));
            NSLGF_TRY(h->tmp3b.ensure((size_t)3 * M * es));
            NSLGF_PROF(h, "curl_masked", s, launch_masked_curl(dt_, U, h->tmp3b.p, 0, (const unsigned char*)h->act_mask.p,
                                                               block, bn[0], bn[1], bn[2], st->dx, s));
            NSLGF_TRY(h->act_w.ensure((size_t)3 * Mn * es));
            NSLGF_TRY(launch_zero(dt_, h->act_w.p, 3 * Mn, s));
            NSLGF_TRY(launch_copy_box(dt_, h->tmp3b.p, bn, soff, h->act_w.p, nn, doff, ext, 3, s));
            NSLGF_TRY(h->act_u[nxt].ensure((size_t)3 * Mn * es));
            NSLGF_TRY(vor2vel(h, h->act_w.p, h->act_u[nxt].p, nn[0], nn[1], nn[2], st->dx, dt_, stream));
            NSLGF_HIP_CHECK(hipStreamSynchronize(s));  // the host mask above is reused
            cur = nxt;
            ++nre;
            nrg += moved ? 1 : 0;
        }
        for (int a = 0; a < 3; ++a) {
            lo[a] = nlo[a];
            hi[a] = nhi[a];
            bn[a] = nn[a];
        }
        ps = gs;
        pn = gn;
        // the step on the box, with D_supp and D_soln in the box's block coordinates
        const int b2[3] = {hi[0] - lo[0], hi[1] - lo[1], hi[2] - lo[2]};
        const long long nb2 = (long long)b2[0] * b2[1] * b2[2];
        std::vector<unsigned char> m2(2 * nb2);
        for (int k = 0; k < b2[2]; ++k)
            for (int j = 0; j < b2[1]; ++j)
                for (int i = 0; i < b2[0]; ++i) {
                    const long long b = ((long long)k * b2[1] + j) * b2[0] + i;
                    m2[b] = gs[gidx(lo[0] + i, lo[1] + j, lo[2] + k)];
                    m2[nb2 + b] = gn[gidx(lo[0] + i, lo[1] + j, lo[2] + k)];
                }
        NSLGF_TRY(h->blockmask.ensure((size_t)2 * nb2));
        NSLGF_HIP_CHECK(hipMemcpyAsync(h->blockmask.p, m2.data(), 2 * nb2, hipMemcpyHostToDevice, s));
        NSLGF_TRY(h->act_d.ensure((size_t)Mn * es));
        NSLGF_TRY(h->act_work.ensure(nslgf_state_bytes(bn[0], bn[1], bn[2], dt_)));
        nslgf_state bs = *st;
        bs.nx = bn[0];
        bs.ny = bn[1];
        bs.nz = bn[2];
        bs.u = h->act_u[cur].p;
        bs.d = h->act_d.p;
        bs.work = h->act_work.p;
        bs.supp_blocks = (const unsigned char*)h->blockmask.p;
        bs.soln_blocks = (const unsigned char*)h->blockmask.p + nb2;
        bs.block = block;
        bs.stage_done = 0;
        const int rc = herk_step(h, &bs, stream);
        st->t = bs.t;
        st->div_max = bs.div_max;
        NSLGF_HIP_CHECK(hipStreamSynchronize(s));  // the host masks are reused by the next step
        NSLGF_TRY(rc);
    }
    // the fields on G: the box's values, zero elsewhere
    const long long MG = (long long)st->nx * st->ny * st->nz;
    const int gd[3] = {st->nx, st->ny, st->nz}, zero[3] = {0, 0, 0};
    const int off[3] = {lo[0] * block, lo[1] * block, lo[2] * block};
    if (nsteps > 0) {
        NSLGF_TRY(launch_zero(dt_, st->u, 3 * MG, s));
        NSLGF_TRY(launch_copy_box(dt_, h->act_u[cur].p, bn, zero, st->u, gd, off, bn, 3, s));
        NSLGF_TRY(launch_zero(dt_, st->d, MG, s));
        NSLGF_TRY(launch_copy_box(dt_, h->act_d.p, bn, zero, st->d, gd, off, bn, 1, s));
    }
    if (reinits) *reinits = nre;
    if (regrids) *regrids = nrg;
    if (box)
        for (int a = 0; a < 3; ++a) {
            box[a] = off[a];
            box[3 + a] = bn[a];
        }
    return NSLGF_OK;
}

int stencil_apply(nslgf_t h, int op, const void* src, void* dst, int ncomp, int nx, int ny, int nz, double dx, int dtype,
                  void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(src && dst && src != dst, "stencil_apply: null or aliased pointers");
    NSLGF_CHECK_ARG(std::isfinite(dx) && dx > 0, "stencil_apply: dx must be > 0");
    NSLGF_CHECK_ARG(op != NSLGF_OP_LAPLACIAN || (ncomp >= 1 && ncomp <= 3), "stencil_apply: ncomp must be 1..3");
    return launch_stencil(op, dtype, src, dst, ncomp, nx, ny, nz, dx, (hipStream_t)stream);
}

int max_cell_speed(nslgf_t h, const void* u, int nx, int ny, int nz, int dtype, double* out, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(u && out, "max_cell_speed: null pointer");
    const int nb = 1024;
    NSLGF_TRY(h->partial.ensure(nb * sizeof(double)));
    hipStream_t s = (hipStream_t)stream;
    NSLGF_TRY(launch_max_speed(dtype, u, nx, ny, nz, (double*)h->partial.p, nb, s));
    std::vector<double> host(nb);
    NSLGF_HIP_CHECK(hipMemcpyAsync(host.data(), h->partial.p, nb * sizeof(double), hipMemcpyDeviceToHost, s));
    NSLGF_HIP_CHECK(hipStreamSynchronize(s));
    double m = 0.0;
    for (double v : host) m = v > m ? v : m;
    *out = m;
    return NSLGF_OK;
}

int nslgf_profile_enable(nslgf_t h, int enable) {
    NSLGF_ENTER(h);
    h->prof.resolve();
    if (enable) {
        h->prof.totals.clear();
        h->prof.order.clear();
    }
    h->prof.on = enable != 0;
    return NSLGF_OK;
}

int nslgf_set_fft_plan(nslgf_t h, int choice) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(choice >= NSLGF_FFT_PLAN_AUTOTUNE && choice <= 2, "nslgf_set_fft_plan: choice must be -2 .. 2");
    h->fft_plan = choice;
    return NSLGF_OK;
}

int nslgf_plan_info(nslgf_t h, int nx, int ny, int nz, int dtype, void* stream, int* vy, int* vz) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(vy && vz, "nslgf_plan_info: null output");
    ConvPlan* p = nullptr;
    NSLGF_TRY(build_plan(h, nx, ny, nz, dtype, (hipStream_t)stream, &p));
    *vy = p->vy;
    *vz = p->vz;
    return NSLGF_OK;
}

int nslgf_copy(nslgf_t h, const void* src, void* dst, size_t n, int dtype, void* stream) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(src && dst && src != dst, "nslgf_copy: null or aliased pointers");
    hipStream_t s = (hipStream_t)stream;
    NSLGF_PROF(h, "copy", s, launch_copy(src, dst, n * dtype_size(dtype), s));
    return NSLGF_OK;
}

int nslgf_set_batch_mode(nslgf_t h, int mode) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(mode == NSLGF_BATCH_PASSES || mode == NSLGF_BATCH_PER_PROBLEM, "nslgf_set_batch_mode: unknown mode");
    if (mode != h->batch_mode) h->batch.reset();
    h->batch_mode = mode;
    return NSLGF_OK;
}

int nslgf_batch_info(nslgf_t h, int* groups, int* launches) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(groups && launches, "nslgf_batch_info: null output");
    *groups = h->batch ? h->batch->groups : 0;
    *launches = h->batch ? h->batch->launches : 0;
    return NSLGF_OK;
}

int nslgf_set_tuning(nslgf_t h, int mode) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(mode == NSLGF_TUNE_DEFAULT || mode == NSLGF_TUNE_AUTO, "nslgf_set_tuning: unknown mode");
    h->tune_mode = mode;
    return NSLGF_OK;
}

int nslgf_tuning_info(nslgf_t h, int nx, int ny, int nz, int dtype, void* stream, int* out) {
    NSLGF_ENTER(h);
    NSLGF_TRY(check_box(nx, ny, nz));
    NSLGF_TRY(check_dtype(dtype));
    NSLGF_CHECK_ARG(out != nullptr, "nslgf_tuning_info: null output");
    hipStream_t s = (hipStream_t)stream;
    ConvPlan* p = nullptr;
    NSLGF_TRY(build_plan(h, nx, ny, nz, dtype, s, &p));
    Tuning tn;
    NSLGF_TRY(get_tuning(h, nx, ny, nz, dtype, s, &tn));
    out[0] = p->vy;
    out[1] = p->vz;
    out[2] = tn.if_rows;
    out[3] = tn.if_seg;
    out[4] = tn.cell_shape;
    return NSLGF_OK;
}

int nslgf_tuning_save(nslgf_t h, const char* path) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(path != nullptr, "nslgf_tuning_save: null path");
    std::string txt = "{\n  \"format\": \"nslgf-tuning-1\",\n  \"entries\": [";
    bool first = true;
    for (const auto& kv : h->tunings) {
        const int nx = std::get<0>(kv.first), ny = std::get<1>(kv.first), nz = std::get<2>(kv.first);
        const int dt = std::get<3>(kv.first);
        const TuneEntry& e = kv.second;
        const Tuning t = e.launch_set ? e.t : default_tuning(nx, ny, nz);
        char line[512];
        std::snprintf(line, sizeof line,
                      "%s\n    {\"nx\": %d, \"ny\": %d, \"nz\": %d, \"dtype\": \"%s\", \"Px\": %d, \"Py\": %d, "
                      "\"Pz\": %d, \"vy\": %d, \"vz\": %d, \"launch\": %d, \"if_rows\": %d, \"if_seg\": %d, "
                      "\"cell_shape\": %d}",
                      first ? "" : ",", nx, ny, nz, dt == NSLGF_F32 ? "f32" : "f64", padded(nx), padded(ny), padded(nz),
                      e.vy, e.vz, e.launch_set ? 1 : 0, t.if_rows, t.if_seg, t.cell_shape);
        txt += line;
        first = false;
    }
    txt += "\n  ]\n}\n";
    FILE* f = std::fopen(path, "w");
    if (!f) {
        set_error(std::string("nslgf_tuning_save: cannot open ") + path);
        return NSLGF_EINVAL;
    }
    const bool ok = std::fwrite(txt.data(), 1, txt.size(), f) == txt.size();
    if (std::fclose(f) != 0 || !ok) {
        set_error(std::string("nslgf_tuning_save: write failed for ") + path);
        return NSLGF_EINVAL;
    }
    return NSLGF_OK;
}

// Reads the integer (or "f32"/"f64" string) value of "key" inside one JSON object's text.
static bool json_field(const std::string& obj, const char* key, int* out) {
    const std::string k = std::string("\"") + key + "\"";
    const size_t at = obj.find(k);
    if (at == std::string::npos) return false;
    size_t p = obj.find(':', at + k.size());
    if (p == std::string::npos) return false;
    ++p;
    while (p < obj.size() && (obj[p] == ' ' || obj[p] == '\t' || obj[p] == '\n')) ++p;
    if (p < obj.size() && obj[p] == '"') {
        const size_t q = obj.find('"', p + 1);
        if (q == std::string::npos) return false;
        const std::string v = obj.substr(p + 1, q - p - 1);
        if (v == "f64") *out = NSLGF_F64;
        else if (v == "f32") *out = NSLGF_F32;
        else return false;
        return true;
    }
    char* end = nullptr;
    const long v = std::strtol(obj.c_str() + p, &end, 10);
    if (end == obj.c_str() + p) return false;
    *out = (int)v;
    return true;
}

int nslgf_tuning_load(nslgf_t h, const char* path) {
    NSLGF_ENTER(h);
    NSLGF_CHECK_ARG(path != nullptr, "nslgf_tuning_load: null path");
    FILE* f = std::fopen(path, "r");
    if (!f) {
        set_error(std::string("nslgf_tuning_load: cannot open ") + path);
        return NSLGF_EINVAL;
    }
    std::string txt;
    char buf[4096];
    size_t got;
    while ((got = std::fread(buf, 1, sizeof buf, f)) > 0) txt.append(buf, got);
    std::fclose(f);
    if (txt.find("\"nslgf-tuning-1\"") == std::string::npos) {
        set_error("nslgf_tuning_load: not an nslgf-tuning-1 file");
        return NSLGF_EINVAL;
    }
    size_t pos = txt.find("\"entries\"");
    if (pos == std::string::npos) {
        set_error("nslgf_tuning_load: no entries");
        return NSLGF_EINVAL;
    }
    std::vector<std::pair<std::tuple<int, int, int, int>, TuneEntry>> read;
    while ((pos = txt.find('{', pos)) != std::string::npos) {
        const size_t end = txt.find('}', pos);
        if (end == std::string::npos) break;
        const std::string obj = txt.substr(pos, end - pos + 1);
        pos = end + 1;
        int nx, ny, nz, dt, Px, Py, Pz, vy, vz, launch, rows, seg, shape;
        if (!(json_field(obj, "nx", &nx) && json_field(obj, "ny", &ny) && json_field(obj, "nz", &nz) &&
              json_field(obj, "dtype", &dt) && json_field(obj, "Px", &Px) && json_field(obj, "Py", &Py) &&
              json_field(obj, "Pz", &Pz) && json_field(obj, "vy", &vy) && json_field(obj, "vz", &vz) &&
              json_field(obj, "launch", &launch) && json_field(obj, "if_rows", &rows) &&
              json_field(obj, "if_seg", &seg) && json_field(obj, "cell_shape", &shape))) {
            set_error("nslgf_tuning_load: an entry lacks a field");
            return NSLGF_EINVAL;
        }
        if (check_box(nx, ny, nz) != NSLGF_OK || check_dtype(dt) != NSLGF_OK || Px != padded(nx) ||
            Py != padded(ny) || Pz != padded(nz) || (rows != 32 && rows != 64 && rows != 128 && rows != 256) ||
            (seg != 16 && seg != 32) || shape < 0 || shape >= kCellShapeCount ||
            (vy >= 0 && !col_variant_valid(Py, dt, vy)) || (vz >= 0 && !col_variant_valid(Pz, dt, vz))) {
            set_error("nslgf_tuning_load: an entry does not fit this library (sizes, padded lengths or choices)");
            return NSLGF_EINVAL;
        }
        TuneEntry e;
        e.t.if_rows = rows;
        e.t.if_seg = seg;
        e.t.cell_shape = shape;
        e.launch_set = launch != 0;
        e.vy = vy;
        e.vz = vz;
        read.emplace_back(std::make_tuple(nx, ny, nz, dt), e);
    }
    // plans built before under the default choice are rebuilt with the loaded variants on next use
    for (const auto& kv : read) {
        h->tunings[kv.first] = kv.second;
        h->plans.erase(std::tuple_cat(kv.first, std::make_tuple(-1)));
    }
    h->batch.reset();
    return NSLGF_OK;
}

int nslgf_profile_read(nslgf_t h, int index, char* name, int name_cap, long long* calls, double* total_ms) {
    NSLGF_ENTER(h);
    h->prof.resolve();
    NSLGF_CHECK_ARG(index >= 0 && index < (int)h->prof.order.size(), "nslgf_profile_read: index out of range");
    const std::string& n = h->prof.order[index];
    const auto& v = h->prof.totals[n];
    if (name && name_cap > 0) {
        std::strncpy(name, n.c_str(), (size_t)name_cap - 1);
        name[name_cap - 1] = 0;
    }
    if (calls) *calls = v.first;
    if (total_ms) *total_ms = v.second;
    return NSLGF_OK;
}

}  // extern "C"
