// Host runtime behind the C ABI of include/llgx.h: workspace and FFT plan,
// demagnetizing-tensor setup, field evaluations, and the explicit stepping
// of Sec. II (Eq. (3)-(6)) with the Eq. (5) controller, the history ring of
// Eq. (6), priming, and HIP-graph replay of fixed steps.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <type_traits>
#include <string>
#include <vector>

#include "batch.hpp"
#include "kernels.hpp"
#include "llgx.h"
#include "tableaux.hpp"

namespace llgx {

static thread_local std::string g_create_error;

// Scratch of llgx_demag_noalloc: one copy per device, held until the process
// ends.  Host code never uses this name as an address: create_ctx resolves
// the device's own address with hipGetSymbolAddress once per device.
static __device__ __align__(256) unsigned char scratch[LLGX_NOALLOC_SCRATCH_BYTES];
static std::mutex g_scratch_mu;
static std::map<int, void*> g_scratch_dev;  // device ordinal -> device address of `scratch`

static int next_pow2(long v) {
    int p = 1;
    while (p < v) p <<= 1;
    return p;
}

// A captured step depends on everything its launches take by value or by
// pointer: the state buffer, the history slots, h (Lagrange weights, stage
// coefficients), the method and order (launch sequence) and the tensor
// generation (N00 inside the per-cell constants, the folded kernel).  A
// graph of nsteps consecutive steps is keyed by the state its first step
// starts from (the others follow from it).
struct GraphKey {
    const void* M;
    int slot0;
    std::vector<int> hist_slots;
    double h;
    int method, p;
    long gen;
    int nsteps = 1;
    bool operator<(const GraphKey& o) const {
        if (nsteps != o.nsteps) return nsteps < o.nsteps;
        if (M != o.M) return M < o.M;
        if (slot0 != o.slot0) return slot0 < o.slot0;
        if (hist_slots != o.hist_slots) return hist_slots < o.hist_slots;
        if (method != o.method) return method < o.method;
        if (p != o.p) return p < o.p;
        if (gen != o.gen) return gen < o.gen;
        return h < o.h;
    }
};

struct Ctx {
    llgx_problem p{};
    int prec = LLGX_F64, spectral = LLGX_SPEC_NATIVE;
    hipStream_t stream = nullptr;
    std::string err;
    size_t tsz = 8;  // bytes per real of the working precision

    // plan
    int nx = 1, ny = 1, nz = 1;
    long ncell = 1;             // cells per sample
    int nb = 1;                 // samples sharing this mesh (batched launches)
    int var[5] = {0, 0, 0, 0, 0};  // launch variant per FFT pass (LLGX_K_XFWD .. LLGX_K_XINV)
    void* hab = nullptr;        // applied field of each sample [nb][3] (device, working precision)
    int Px = 1, Py = 1, Pz = 1, LX = 0, Kx = 1, SX = 16, Kyf = 1, Kzf = 1;

    // device workspace
    void* kfold = nullptr;
    void* specA = nullptr;
    void* specB = nullptr;
    std::map<int, void*> tw_work;  // twiddle tables in the working precision
    std::map<int, void*> tw_f64;   // twiddle tables in double (tensor setup)
    void* M = nullptr;
    void* Mnew = nullptr;
    void* Mk = nullptr;
    void* Mk2 = nullptr;        // second stage-input buffer (chained stages ping-pong)
    void* F[MAX_F] = {};
    void* G[MAX_HIST] = {};
    void* E[MAX_F] = {};        // Eq. (6) fields at the distinct sub-step times of a step
    // Mk2 and the first E fields may live inside spectrum B (see create_ctx);
    // those are not freed on their own
    bool mk2_in_b = false;
    bool e_in_b[MAX_F] = {};
    double* parts = nullptr;
    int nparts = 1;             // blocks of the 1-D reduction kernels
    long nparts_alloc = 1;      // capacity of parts (also covers the 2-D cell grid)
    double* scal = nullptr;     // [0] error norm, [1..3] sums for <M>
    int* empty_flag = nullptr;  // device: [0] some cell of M has M = 0; [1] the same for the
                                // input of a field call (llgx_demag / heff / rhs)
    bool field_input = false;   // phys() reads flag [1] (during a field call)
    const int* empty_use = nullptr;  // when set, phys() reads this flag instead
    void* spec_use[2] = {nullptr, nullptr};  // when set, the spectra A and B of the passes
    void* noalloc = nullptr;    // device address of this device's llgx_demag_noalloc scratch
    double* octant = nullptr;   // real-space tensor for offsets 0..n-1 (double)
    bool have_kernel = false;
    long kernel_gen = 0;        // bumped whenever the tensor (and N00) changes
    bool have_m = false;
    double n00[3] = {0, 0, 0};

    // stepping state
    double t = 0.0, h_next = 0.0;
    struct Hist {
        double t;
        int slot;
    };
    std::vector<Hist> hist;  // previous accepted iterations, oldest first
    bool fsal_valid = false;
    // ABM2: F_n (in F[0]) and its stored field (slot abm_slot) at (t, M);
    // F_{n-1} (in F[2]) and h_{n-1}
    bool abm_have_f = false, abm_have_prev = false;
    double abm_hprev = 0.0;
    int abm_slot = 0;
    int cur_method = -1, cur_p = -100;
    long long n_exact = 0, n_extrap = 0, n_acc = 0, n_rej = 0, n_forced = 0;

    std::map<GraphKey, hipGraphExec_t> graphs;

    // When set, the launches of one step attempt are recorded here (kind of
    // the job-table batched kernel, its template count, its arguments)
    // instead of made; rec_unsupported is set by a launch that has no
    // job-table form (16-bit spectra, error-norm reduction, ...).
    struct Rec {
        int kind, nf;
        std::vector<unsigned char> arg;
    };
    std::vector<Rec>* rec = nullptr;
    bool rec_unsupported = false;

    // per-kernel event timing (eager launches only)
    bool prof = false;
    struct Mark {
        int kind;
        hipEvent_t a, b;
    };
    std::vector<Mark> marks;
    std::vector<hipEvent_t> spare;
    int open_kind = -1;

    llgx_status fail(llgx_status code, const char* fmt, ...) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        err = buf;
        return code;
    }
};

#define HIPCHK(ctx, expr)                                                                                   \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return (ctx)->fail(e_ == hipErrorOutOfMemory ? LLGX_E_OOM : LLGX_E_HIP, "%s failed: %s (%s:%d)", \
                               #expr, hipGetErrorString(e_), __FILE__, __LINE__);                           \
    } while (0)

static llgx_status dalloc(Ctx* c, void** p, size_t bytes) {
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        *p = nullptr;
        return c->fail(e == hipErrorOutOfMemory ? LLGX_E_OOM : LLGX_E_HIP, "hipMalloc(%zu) failed: %s", bytes,
                       hipGetErrorString(e));
    }
    return LLGX_OK;
}

static hipEvent_t take_event(Ctx* c) {
    if (!c->spare.empty()) {
        hipEvent_t e = c->spare.back();
        c->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
    return e;
}

// bracket the next launch with events when profiling
struct ProfScope {
    Ctx* c;
    hipEvent_t a = nullptr;
    int kind;
    ProfScope(Ctx* c_, int kind_) : c(c_), kind(kind_) {
        if (c->prof) {
            a = take_event(c);
            if (a) (void)hipEventRecord(a, c->stream);
        }
    }
    ~ProfScope() {
        if (a) {
            hipEvent_t b = take_event(c);
            if (b) {
                (void)hipEventRecord(b, c->stream);
                c->marks.push_back({kind, a, b});
            } else {
                c->spare.push_back(a);
            }
        }
    }
};

#define PROF(kind) ProfScope prof_scope_(c, kind)

// twiddle table e^{-2 pi i m/L}, m < L, built in double
template <typename T>
static llgx_status make_table(Ctx* c, std::map<int, void*>& tabs, int L) {
    if (L < 2 || tabs.count(L)) return LLGX_OK;
    std::vector<T> h(2 * (size_t)L);
    for (int m = 0; m < L; ++m) {
        const double a = 2.0 * M_PI * (double)m / (double)L;
        h[2 * m] = (T)std::cos(a);
        h[2 * m + 1] = (T)(-std::sin(a));
    }
    void* d = nullptr;
    llgx_status st = dalloc(c, &d, h.size() * sizeof(T));
    if (st) return st;
    HIPCHK(c, hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
    tabs[L] = d;
    return LLGX_OK;
}

template <typename T>
static const cx<T>* table(Ctx* c, int L, bool f64) {
    auto& tabs = f64 ? c->tw_f64 : c->tw_work;
    auto it = tabs.find(L);
    return it == tabs.end() ? nullptr : (const cx<T>*)it->second;
}

template <typename T>
static Phys<T> phys(const Ctx* c) {
    const llgx_problem& p = c->p;
    const double mu0 = 4e-7 * M_PI;
    const double exf = 2.0 * p.A / (mu0 * p.Ms * p.Ms);
    Phys<T> ph;
    ph.exx = (T)(exf / (p.dx * p.dx));
    ph.exy = (T)(exf / (p.dy * p.dy));
    ph.exz = (T)(exf / (p.dz * p.dz));
    ph.ani = (T)(2.0 * p.K / (mu0 * p.Ms * p.Ms));
    double un = std::sqrt(p.easy[0] * p.easy[0] + p.easy[1] * p.easy[1] + p.easy[2] * p.easy[2]);
    for (int i = 0; i < 3; ++i) {
        ph.u[i] = (T)(un > 0 ? p.easy[i] / un : 0.0);
        ph.n00[i] = (T)c->n00[i];
    }
    const double gp = p.gamma / (1.0 + p.alpha * p.alpha);
    ph.gp = (T)gp;
    ph.gpa = (T)(gp * p.alpha / p.Ms);
    ph.nx = c->nx;
    ph.ny = c->ny;
    ph.nz = c->nz;
    ph.nb = c->nb;
    ph.hab = (const T*)c->hab;
    ph.empty = c->empty_use ? c->empty_use : c->empty_flag + (c->field_input ? 1 : 0);
    return ph;
}

template <typename T>
static Combo<T> plain(const void* base) {
    Combo<T> cb{};
    cb.base = (const T*)base;
    cb.nf = 0;
    return cb;
}

// Recompute an empty-cell flag (slot 0: from the state M; slot 1: from the
// input of a field call) on the stream, with no host synchronisation.
static llgx_status detect_empty(Ctx* c, const void* M = nullptr, int slot = 0) {
    int* flag = c->empty_flag + slot;
    if (!M) M = c->M;
    HIPCHK(c, hipMemsetAsync(flag, 0, sizeof(int), c->stream));
    if (c->prec == LLGX_F32)
        HIPCHK(c, launch_detect_empty<float>(c->stream, c->ncell, c->nb, (const float*)M, flag));
    else
        HIPCHK(c, launch_detect_empty<double>(c->stream, c->ncell, c->nb, (const double*)M, flag));
    return LLGX_OK;
}

// ---------------------------------------------------------------------------
// one exact evaluation of Eq. (2) on the stage input `in` (Eq. (4)), ending
// in the inverse x pass selected by `mode`.  Spectra stored as S; with 16-bit
// storage the transforms are scaled so that every stored spectrum is O(1):
// the x pass takes M/(Ms Px), the y pass stores 1/Py of its output, the
// kernel product carries Px Py (so it applies -N^/Pz), and the field is
// multiplied by Ms when it is formed.  With S = T every scale is 1.
template <typename T>
struct EvalArgs {
    Combo<T> in;
    T* mk_out;
    int mode;
    const T* Mrhs;
    XinvOut out;
};

template <typename A>
static void record(Ctx* c, int kind, int nf, const A& a) {
    Ctx::Rec r{kind, nf, std::vector<unsigned char>(sizeof(A))};
    std::memcpy(r.arg.data(), &a, sizeof(A));
    c->rec->push_back(std::move(r));
}

// the arguments of pass `kind` for the job-table batched kernels
template <typename T>
static void record_pass(Ctx* c, int kind, const EvalArgs<T>& a, void* A, void* B) {
    using C = cx<T>;
    const C* twL = table<T>(c, c->LX, false);
    const C* twP = table<T>(c, c->Px, false);
    const long sa = (long)c->nz * c->ny * c->SX, sb = (long)c->nz * c->Py * c->SX;
    switch (kind) {
        case LLGX_K_XFWD:
            record(c, BK_XFWD, 0,
                   BXfwd<T>{a.in, a.mk_out, c->nx, 3L * c->ny * c->nz * c->nb, (C*)A, c->SX, twL, twP, c->LX, 0});
            break;
        case LLGX_K_YFWD:
            record(c, BK_COL, 0,
                   BCol<T>{(const C*)A, sa, (long)c->ny * c->SX, c->SX, c->ny, (C*)B, sb, (long)c->Py * c->SX, c->SX,
                           c->Py, c->Kx, table<T>(c, c->Py, false), c->Py, c->nz, 3 * c->nb, 0, 0});
            break;
        case LLGX_K_ZMUL:
            record(c, BK_ZMUL, 0,
                   BZmul<T>{(C*)(c->Py > 1 ? B : A), c->SX, c->Kx, c->nz, c->Py > 1 ? c->Py : c->ny, c->Py, c->nb,
                            (const T*)c->kfold, table<T>(c, c->Pz, false), c->Pz, 0, 0, 0});
            break;
        case LLGX_K_YINV:
            record(c, BK_COL, 1,
                   BCol<T>{(const C*)B, sb, (long)c->Py * c->SX, c->SX, c->Py, (C*)A, sa, (long)c->ny * c->SX, c->SX,
                           c->ny, c->Kx, table<T>(c, c->Py, false), c->Py, c->nz, 3 * c->nb, 0, 0});
            break;
        case LLGX_K_XINV:
            if (a.mode != XINV_RHS) {
                c->rec_unsupported = true;
                break;
            }
            record(c, BK_XINV, 0, BXinv<T>{(const C*)A, c->SX, a.Mrhs, phys<T>(c), a.out, twL, twP, c->LX, 0, 0});
            break;
    }
}

static bool pass_exists(const Ctx* c, int kind) {
    return !((kind == LLGX_K_YFWD || kind == LLGX_K_YINV) && c->Py == 1);
}

// launch one pass (kind LLGX_K_XFWD .. LLGX_K_XINV) with the handle's variant
template <typename T, typename S>
static llgx_status run_pass(Ctx* c, int kind, const EvalArgs<T>& a) {
    hipStream_t s = c->stream;
    void* A = c->spec_use[0] ? c->spec_use[0] : c->specA;
    void* B = c->spec_use[1] ? c->spec_use[1] : c->specB;
    const cx<T>* twL = table<T>(c, c->LX, false);
    const cx<T>* twP = table<T>(c, c->Px, false);
    const bool native = std::is_same<T, S>::value;
    const long sa = (long)c->nz * c->ny * c->SX, sb = (long)c->nz * c->Py * c->SX;
    if (c->rec) {
        if constexpr (std::is_same<T, S>::value)
            record_pass<T>(c, kind, a, A, B);
        else
            c->rec_unsupported = true;
        return LLGX_OK;
    }
    switch (kind) {
        case LLGX_K_XFWD: {
            const T fscale = native ? T(1) : (T)(1.0 / (c->p.Ms * c->Px));
            HIPCHK(c, (launch_xfwd<T, S>(s, c->LX, a.in, a.mk_out, c->nx, 3L * c->ny * c->nz * c->nb, A, c->SX, twL,
                                         twP, fscale, c->var[kind])));
            break;
        }
        case LLGX_K_YFWD: {
            const T yscale = native ? T(1) : (T)(1.0 / c->Py);
            HIPCHK(c, (launch_colfft<T, S>(s, c->Py, false, A, sa, (long)c->ny * c->SX, c->SX, c->ny, B, sb,
                                           (long)c->Py * c->SX, c->SX, c->Py, c->Kx, c->nz, 3 * c->nb,
                                           table<T>(c, c->Py, false), yscale, c->var[kind])));
            break;
        }
        case LLGX_K_ZMUL: {
            void* work = c->Py > 1 ? B : A;
            const int nyrows = c->Py > 1 ? c->Py : c->ny;
            HIPCHK(c, (launch_zmul<T, S>(s, c->Pz, work, c->SX, c->Kx, c->nz, nyrows, c->Py, c->Pz,
                                         (const T*)c->kfold, c->Kyf, c->Kzf, table<T>(c, c->Pz, false), c->nb,
                                         c->var[kind])));
            break;
        }
        case LLGX_K_YINV:
            HIPCHK(c, (launch_colfft<T, S>(s, c->Py, true, B, sb, (long)c->Py * c->SX, c->SX, c->Py, A, sa,
                                           (long)c->ny * c->SX, c->SX, c->ny, c->Kx, c->nz, 3 * c->nb,
                                           table<T>(c, c->Py, false), T(1), c->var[kind])));
            break;
        case LLGX_K_XINV: {
            const T hscale = native ? T(1) : (T)c->p.Ms;
            HIPCHK(c, (launch_xinv<T, S>(s, c->LX, a.mode, A, c->SX, a.Mrhs, phys<T>(c), a.out, twL, twP, hscale,
                                         c->var[kind])));
            break;
        }
        default:
            return c->fail(LLGX_E_ARG, "unknown pass %d", kind);
    }
    return LLGX_OK;
}

template <typename T, typename S>
static llgx_status eval_exact_s(Ctx* c, const Combo<T>& in, T* mk_out, int mode, const T* Mrhs, const XinvOut& out) {
    const EvalArgs<T> a{in, mk_out, mode, Mrhs, out};
    for (int kind = LLGX_K_XFWD; kind <= LLGX_K_XINV; ++kind) {
        if (!pass_exists(c, kind)) {
            // a group without y passes takes no jobs of the batch's y launches
            if (c->rec) record(c, BK_COL, kind == LLGX_K_YINV ? 1 : 0, BCol<T>{});
            continue;
        }
        PROF(kind);
        llgx_status st = run_pass<T, S>(c, kind, a);
        if (st) return st;
    }
    return LLGX_OK;
}

// Average duration of `reps` back-to-back launches of one pass with
// variant v, between two HIP events on the handle's stream.  Works on the
// spectral workspace and the stage-input scratch array only (x pass from M,
// inverse x pass into M_k), so the stepping state is left as it was.
template <typename T, typename S>
static llgx_status time_pass(Ctx* c, int kind, int v, int reps, double* us) {
    const EvalArgs<T> a{plain<T>(c->M), nullptr, XINV_RHS, (const T*)c->M, XinvOut{nullptr, c->Mk, nullptr}};
    const int saved = c->var[kind];
    c->var[kind] = v;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    llgx_status st = LLGX_OK;
    if (hipEventCreateWithFlags(&e0, hipEventDisableSystemFence) != hipSuccess ||
        hipEventCreateWithFlags(&e1, hipEventDisableSystemFence) != hipSuccess)
        st = c->fail(LLGX_E_HIP, "hipEventCreate failed");
    for (int w = 0; w < 2 && st == LLGX_OK; ++w) st = run_pass<T, S>(c, kind, a);
    if (st == LLGX_OK && hipEventRecord(e0, c->stream) != hipSuccess) st = c->fail(LLGX_E_HIP, "hipEventRecord failed");
    for (int r = 0; r < reps && st == LLGX_OK; ++r) st = run_pass<T, S>(c, kind, a);
    if (st == LLGX_OK && hipEventRecord(e1, c->stream) != hipSuccess) st = c->fail(LLGX_E_HIP, "hipEventRecord failed");
    float ms = 0.f;
    if (st == LLGX_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        st = c->fail(LLGX_E_HIP, "event timing failed");
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    c->var[kind] = saved;
    if (st == LLGX_OK) *us = 1e3 * (double)ms / reps;
    return st;
}

template <typename T>
static llgx_status eval_exact(Ctx* c, const Combo<T>& in, T* mk_out, int mode, const T* Mrhs, const XinvOut& out) {
    if constexpr (std::is_same<T, float>::value) {
        if (c->spectral == LLGX_SPEC_BF16) return eval_exact_s<float, __bf16>(c, in, mk_out, mode, Mrhs, out);
        if (c->spectral == LLGX_SPEC_F16) return eval_exact_s<float, _Float16>(c, in, mk_out, mode, Mrhs, out);
    }
    return eval_exact_s<T, T>(c, in, mk_out, mode, Mrhs, out);
}

// ---------------------------------------------------------------------------
// demagnetizing tensor -> folded real k-space kernel (double FFT passes)
template <typename T>
static llgx_status kernel_from_octant_or_real(Ctx* c, const std::vector<double>* full_host) {
    hipStream_t s = c->stream;
    const long preal = (long)c->Pz * c->Py * c->Px;
    const long pspec = (long)c->Pz * c->Py * c->SX;
    void* real = nullptr;
    void* spec = nullptr;
    llgx_status st = dalloc(c, &real, preal * sizeof(double));
    if (st) return st;
    st = dalloc(c, &spec, pspec * 2 * sizeof(double));
    if (st) {
        (void)hipFree(real);
        return st;
    }
    if (!c->kfold) {
        st = dalloc(c, &c->kfold, 6L * c->Kzf * c->Kyf * c->SX * sizeof(T));
        if (st) {
            (void)hipFree(real);
            (void)hipFree(spec);
            return st;
        }
        HIPCHK(c, hipMemsetAsync(c->kfold, 0, 6L * c->Kzf * c->Kyf * c->SX * sizeof(T), s));
    }
    for (int L : {c->LX, c->Px, c->Py, c->Pz}) {
        st = make_table<double>(c, c->tw_f64, L);
        if (st) return st;
    }
    // K^ = -N^ / (Px Py Pz); with 16-bit spectra (scaled by 1/(Px Py) in the x
    // and y passes) the kernel also carries Px Py, a power of two, so the
    // fold's rounding is unchanged
    const bool native_spec = c->spectral == LLGX_SPEC_NATIVE;
    const double scale = native_spec ? -1.0 / ((double)c->Px * c->Py * c->Pz) : -1.0 / (double)c->Pz;
    std::vector<double> hreal;
    for (int comp = 0; comp < 6; ++comp) {
        if (full_host) {
            // caller's tensor at wrap-around indices of the padded grid
            hreal.assign(preal, 0.0);
            const int fx = 2 * c->nx - 1, fy = 2 * c->ny - 1, fz = 2 * c->nz - 1;
            for (int dz = -(c->nz - 1); dz < c->nz; ++dz)
                for (int dy = -(c->ny - 1); dy < c->ny; ++dy)
                    for (int dx = -(c->nx - 1); dx < c->nx; ++dx) {
                        const long src = (((long)comp * fz + dz + c->nz - 1) * fy + dy + c->ny - 1) * fx + dx + c->nx - 1;
                        const int pz = (dz + c->Pz) % c->Pz, py = (dy + c->Py) % c->Py, px = (dx + c->Px) % c->Px;
                        hreal[((long)pz * c->Py + py) * c->Px + px] = (*full_host)[src];
                    }
            HIPCHK(c, hipMemcpyAsync(real, hreal.data(), preal * sizeof(double), hipMemcpyHostToDevice, s));
        } else {
            HIPCHK(c, hipMemsetAsync(real, 0, preal * sizeof(double), s));
            HIPCHK(c, launch_scatter_tensor(s, c->octant, comp, c->nx, c->ny, c->nz, c->Px, c->Py, c->Pz,
                                            (double*)real));
        }
        cx<double>* sp = (cx<double>*)spec;
        HIPCHK(c, (launch_xfwd<double, double>(s, c->LX, plain<double>(real), nullptr, c->Px, (long)c->Pz * c->Py, sp,
                                               c->SX, table<double>(c, c->LX, true), table<double>(c, c->Px, true),
                                               1.0, 0)));
        if (c->Py > 1)
            HIPCHK(c, (launch_colfft<double, double>(s, c->Py, false, sp, 0, (long)c->Py * c->SX, c->SX, c->Py, sp, 0,
                                                     (long)c->Py * c->SX, c->SX, c->Py, c->Kx, c->Pz, 1,
                                                     table<double>(c, c->Py, true), 1.0, 0)));
        if (c->Pz > 1)
            HIPCHK(c, (launch_colfft<double, double>(s, c->Pz, false, sp, 0, c->SX, (long)c->Py * c->SX, c->Pz, sp, 0,
                                                     c->SX, (long)c->Py * c->SX, c->Pz, c->Kx, c->Py, 1,
                                                     table<double>(c, c->Pz, true), 1.0, 0)));
        HIPCHK(c, launch_fold<T>(s, sp, c->SX, c->Kx, c->Py, c->Pz, c->Kyf, c->Kzf, scale, comp, (T*)c->kfold,
                                 c->parts, c->nparts));
    }
    HIPCHK(c, hipStreamSynchronize(s));
    (void)hipFree(real);
    (void)hipFree(spec);
    c->have_kernel = true;
    // graphs captured with the previous tensor are never replayed again
    c->kernel_gen++;
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    return LLGX_OK;
}

static llgx_status precompute(Ctx* c) {
    hipStream_t s = c->stream;
    if (!c->octant) {
        llgx_status st = dalloc(c, (void**)&c->octant, 6L * c->ncell * sizeof(double));
        if (st) return st;
    }
    HIPCHK(c, launch_newell_octant(s, c->nx, c->ny, c->nz, c->p.dx, c->p.dy, c->p.dz, c->octant));
    double n00[3];
    for (int i = 0; i < 3; ++i)
        HIPCHK(c, hipMemcpyAsync(&n00[i], c->octant + (long)i * c->ncell, sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipStreamSynchronize(s));
    for (int i = 0; i < 3; ++i) c->n00[i] = n00[i];
    llgx_status st = c->prec == LLGX_F32 ? kernel_from_octant_or_real<float>(c, nullptr)
                                         : kernel_from_octant_or_real<double>(c, nullptr);
    return st;
}

// ---------------------------------------------------------------------------
// stepping
static int extrap_order(const Tableau* tab, int extrap) {
    return extrap == LLGX_EXTRAP_MATCHED ? tab->order : extrap;
}

static std::vector<double> lagrange(const std::vector<double>& nodes, double t) {
    std::vector<double> w(nodes.size());
    for (size_t i = 0; i < nodes.size(); ++i) {
        double li = 1.0;
        for (size_t j = 0; j < nodes.size(); ++j)
            if (j != i) li *= (t - nodes[j]) / (nodes[i] - nodes[j]);
        w[i] = li;
    }
    return w;
}

// Host-side decisions of one attempt (pointers, slots, weights), so that the
// same enqueue can run eagerly or be captured into a graph.
struct Plan {
    const Tableau* tab;
    int p;            // -1: full evaluation
    bool extrap;      // Eq. (6) used at stages >= 2
    bool stage1;      // stage 1 must be evaluated (not FSAL reuse, not a retry)
    int slot0;        // G slot receiving this iteration's stored field
    double h;
    bool want_err;
    bool in_place;    // Eq. (3) update written over M0 (fixed steps: no retry needs M0)
};

template <typename T>
static llgx_status enqueue_attempt(Ctx* c, const Plan& pl) {
    const Tableau* tab = pl.tab;
    const double h = pl.h;
    // Stage j reads M_j = M0 + h sum_l a_jl F_l (Eq. 4).  When row j holds only
    // a_j,j-1 (RK4), the kernel that forms F_{j-1} also writes M_j, into one of
    // two buffers taken in turn (the stencil of stage j-1 still reads M_{j-1}).
    auto chained = [&](int j) {
        if (!pl.extrap || j < 1 || j >= tab->S || tab->a[j][j - 1] == 0.0) return false;
        for (int l = 0; l + 1 < j; ++l)
            if (tab->a[j][l] != 0.0) return false;
        return true;
    };
    auto mkbuf = [&](int j) { return (j & 1) ? c->Mk : c->Mk2; };
    std::vector<bool> formed(tab->S, false);
    if (pl.stage1) {
        XinvOut out{nullptr, c->F[0], pl.p >= 0 ? c->G[pl.slot0] : nullptr, nullptr, 0.0};
        if (chained(1)) {
            out.mnext = mkbuf(1);
            out.cnext = h * tab->a[1][0];
            formed[1] = true;
        }
        llgx_status st = eval_exact<T>(c, plain<T>(c->M), nullptr, XINV_RHS, (const T*)c->M, out);
        if (st) return st;
    }
    std::vector<double> nodes;
    std::vector<int> slots;
    // distinct sub-step times of stages 2..S: field index per stage
    std::vector<double> times;
    std::vector<int> field_of(tab->S, -1);
    bool fuse_ep = false;
    EPoly<T> ep_fused{};
    if (pl.extrap) {
        for (auto& hh : c->hist) {
            nodes.push_back(hh.t - c->t);
            slots.push_back(hh.slot);
        }
        nodes.push_back(0.0);
        slots.push_back(pl.slot0);
        for (int k = 1; k < tab->S; ++k) {
            if (pl.p == 0 || tab->c[k] == 0.0) continue;  // G0 itself
            int j = -1;
            for (size_t q = 0; q < times.size(); ++q)
                if (times[q] == tab->c[k]) j = (int)q;
            if (j < 0) {
                j = (int)times.size();
                times.push_back(tab->c[k]);
            }
            field_of[k] = j;
        }
        if (!times.empty()) {
            EPoly<T> ep{};
            ep.ng = (int)nodes.size();
            ep.nd = (int)times.size();
            for (int i = 0; i < ep.ng; ++i) ep.g[i] = (const T*)c->G[slots[i]];
            for (int j = 0; j < ep.nd; ++j) {
                const std::vector<double> w = lagrange(nodes, times[j] * h);
                for (int i = 0; i < ep.ng; ++i) ep.w[j][i] = (T)w[i];
                ep.out[j] = (T*)c->E[j];
            }
            // with at most two distinct times, the first extrapolated stage
            // (not the last) forms the Eq. (6) fields itself
            fuse_ep = !c->rec && ep.nd <= 2 && ep.ng <= 6 && tab->S >= 3;
            if (fuse_ep) {
                ep_fused = ep;
            } else {
                PROF(LLGX_K_EPOLY);
                if (c->rec)
                    record(c, BK_EPOLY, ep.ng, BEpoly<T>{ep, 3 * c->ncell * c->nb});
                else
                    HIPCHK(c, launch_epoly<T>(c->stream, 3 * c->ncell * c->nb, ep));
            }
        }
    }
    // Eq. (3) operands: stage derivatives used by the update or by the estimate
    Final<T> fs{};
    fs.err = pl.want_err && tab->order_hat > 0;
    auto add_final = [&](int k) {
        const bool use_e = fs.err && tab->b[k] != tab->bh[k];
        fs.f[fs.n] = (const T*)c->F[k];
        fs.cb[fs.n] = (T)(h * tab->b[k]);
        fs.ce[fs.n] = use_e ? h * (tab->b[k] - tab->bh[k]) : 0.0;
        fs.n++;
    };
    for (int k = 0; k < tab->S; ++k) {
        const bool last_fused = pl.extrap && k == tab->S - 1;
        if (last_fused) break;
        const bool use_b = tab->b[k] != 0.0;
        const bool use_e = fs.err && tab->b[k] != tab->bh[k];
        if (use_b || use_e) add_final(k);
    }
    bool fused_final = false;
    for (int k = 1; k < tab->S; ++k) {
        Combo<T> cb{};
        cb.base = (const T*)c->M;
        cb.nf = 0;
        for (int l = 0; l < k; ++l) {
            if (tab->a[k][l] == 0.0) continue;
            cb.f[cb.nf] = (const T*)c->F[l];
            cb.coef[cb.nf] = (T)(h * tab->a[k][l]);
            cb.nf++;
        }
        if (pl.extrap) {
            if (formed[k]) {
                cb = plain<T>(mkbuf(k));
            } else if (cb.nf > 0) {
                // form M_k once instead of at every stencil read
                PROF(LLGX_K_COMBINE);
                if (c->rec)
                    record(c, BK_COMBINE, cb.nf, BCombine<T>{cb, (T*)mkbuf(k), 3 * c->ncell * c->nb});
                else
                    HIPCHK(c, launch_combine<T>(c->stream, 3 * c->ncell * c->nb, cb, (T*)mkbuf(k)));
                cb = plain<T>(mkbuf(k));
            }
            Extrap<T> ex{};
            ex.n = 1;
            ex.w[0] = T(1);
            ex.g[0] = field_of[k] < 0 ? (const T*)c->G[pl.slot0] : (const T*)c->E[field_of[k]];
            const bool with_ep = fuse_ep && k == 1;
            ProfScope ps(c, k == tab->S - 1 ? LLGX_K_FINAL : with_ep ? LLGX_K_EPOLY : LLGX_K_EXTRAP);
            if (k == tab->S - 1) {
                add_final(k);  // own derivative, last entry
                T* mnew = (T*)(pl.in_place ? c->M : c->Mnew);
                if (c->rec)
                    record(c, BK_STAGE_FINAL, fs.n,
                           BStageFinal<T>{cb, ex, phys<T>(c), (const T*)c->M, fs, 1.0 / c->p.Ms, mnew, c->parts});
                else
                    HIPCHK(c, launch_stage_final<T>(c->stream, cb, ex, phys<T>(c), (const T*)c->M, fs,
                                                    1.0 / c->p.Ms, mnew, c->parts));
                fused_final = true;
            } else {
                NextStage<T> nx{nullptr, nullptr, T(0)};
                if (chained(k + 1)) {
                    nx = NextStage<T>{(const T*)c->M, (T*)mkbuf(k + 1), (T)(h * tab->a[k + 1][k])};
                    formed[k + 1] = true;
                }
                if (c->rec)
                    record(c, BK_STAGE, 0, BStage<T>{cb, ex, phys<T>(c), (T*)c->F[k], nx});
                else if (with_ep)
                    HIPCHK(c, launch_stage_ep<T>(c->stream, cb, ex, ep_fused, field_of[k], phys<T>(c), (T*)c->F[k],
                                                 nx));
                else
                    HIPCHK(c, launch_extrap_rhs<T>(c->stream, cb, ex, phys<T>(c), (T*)c->F[k], nx));
            }
        } else {
            XinvOut out{nullptr, c->F[k], nullptr};
            llgx_status st = eval_exact<T>(c, cb, (T*)c->Mk, XINV_RHS, (const T*)c->Mk, out);
            if (st) return st;
        }
    }
    int nred = c->nparts;
    if (fused_final) {
        nred = (int)cell_grid(c->nx, c->ny, c->nz, c->nb).nblocks;
    } else {
        PROF(LLGX_K_FINAL);
        T* mnew = (T*)(pl.in_place ? c->M : c->Mnew);
        if (c->rec)
            record(c, BK_FINAL, fs.n,
                   BFinal<T>{c->ncell, c->nb, (const T*)c->M, fs, 1.0 / c->p.Ms, mnew, c->parts, c->nparts});
        else
            HIPCHK(c, launch_final<T>(c->stream, c->ncell, c->nb, (const T*)c->M, fs, 1.0 / c->p.Ms, mnew, c->parts,
                                      c->nparts));
    }
    if (pl.want_err) {
        PROF(LLGX_K_OTHER);
        if (c->rec)
            c->rec_unsupported = true;
        else
            HIPCHK(c, launch_reduce_max(c->stream, c->parts, nred, c->scal));
    }
    return LLGX_OK;
}

static int free_slot(const Ctx* c) {
    for (int s = 0; s < MAX_HIST; ++s) {
        bool used = false;
        for (auto& hh : c->hist) used |= hh.slot == s;
        if (!used) return s;
    }
    return -1;
}

template <typename T>
static llgx_status commit(Ctx* c, const Plan& pl, double h_used) {
    if (pl.p > 0) {
        c->hist.push_back({c->t, pl.slot0});
        while ((int)c->hist.size() > pl.p) c->hist.erase(c->hist.begin());
    }
    if (!pl.in_place) std::swap(c->M, c->Mnew);
    c->fsal_valid = false;
    if (pl.p < 0 && pl.tab->fsal) {
        // the last stage was evaluated at the accepted M: it is stage 1 of the next step
        std::swap(c->F[0], c->F[pl.tab->S - 1]);
        c->fsal_valid = true;
    }
    c->t += h_used;
    c->n_acc++;
    return LLGX_OK;
}

static llgx_status check_stepper(Ctx* c, const llgx_stepper* s, const Tableau** tab, int* p) {
    if (!s) return c->fail(LLGX_E_ARG, "null stepper");
    *tab = tableau_for(s->method);
    if (!*tab) return c->fail(LLGX_E_ARG, "unknown method %d", s->method);
    *p = extrap_order(*tab, s->extrap);
    if (*p < -1 || *p > MAX_HIST - 1) return c->fail(LLGX_E_ARG, "extrapolation order %d out of range", s->extrap);
    if (s->adaptive && (*tab)->order_hat == 0) return c->fail(LLGX_E_ARG, "%s has no embedded estimate", (*tab)->name);
    if (!(s->h > 0)) return c->fail(LLGX_E_ARG, "h must be > 0");
    if (!c->have_kernel) return c->fail(LLGX_E_STATE, "demag kernel not computed (llgx_precompute_demag)");
    if (!c->have_m) return c->fail(LLGX_E_STATE, "magnetization not set (llgx_set_m)");
    if (s->method != c->cur_method || *p != c->cur_p) {
        c->hist.clear();
        c->fsal_valid = false;
        c->abm_have_f = c->abm_have_prev = false;
        c->cur_method = s->method;
        c->cur_p = *p;
        c->h_next = 0.0;
    }
    if (s->renormalize) c->fsal_valid = false;
    return LLGX_OK;
}

// max over cells of |dM/dt| / Ms of the derivative in F[0] (the first
// stage's, at the state the step starts from), read back to the host
template <typename T>
static llgx_status read_max_dmdt(Ctx* c, double* out) {
    {
        PROF(LLGX_K_OTHER);
        HIPCHK(c, launch_max_norm<T>(c->stream, c->ncell, c->nb, (const T*)c->F[0], 1.0 / c->p.Ms, c->parts,
                                     c->nparts));
    }
    {
        PROF(LLGX_K_OTHER);
        HIPCHK(c, launch_reduce_max(c->stream, c->parts, c->nparts, c->scal + 4));
    }
    HIPCHK(c, hipMemcpyAsync(out, c->scal + 4, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LLGX_OK;
}

// One accepted ABM2 step (PECE, ref. [32]):
//   P: M_p = M_n + h ((1 + r/2) F_n - (r/2) F_{n-1}), r = h / h_{n-1}
//      (M_n + h F_n, Heun's predictor, when no F_{n-1} is held)
//   E: F_p at (t_n + h, M_p), by Eq. (6) once the history is primed
//   C: M_{n+1} = M_n + (h/2)(F_n + F_p)
//   E: F_{n+1} at (t_{n+1}, M_{n+1}) with exact Eq. (2), after acceptance
// e = k(r) max |M_{n+1} - M_p| / Ms with the Milne factor k = r / (3 (r + 1))
// (1 on the starting Heun step).  The exact evaluation's stored field is the
// next iteration's start node of Eq. (6).
template <typename T>
static llgx_status do_step_abm(Ctx* c, const llgx_stepper* s, int p, llgx_step_info* info) {
    const long long ex0 = c->n_exact, xt0 = c->n_extrap;
    if (!c->abm_have_f) {
        const int slot = free_slot(c);
        XinvOut out{nullptr, c->F[0], p >= 0 ? c->G[slot] : nullptr, nullptr, 0.0};
        llgx_status st = eval_exact<T>(c, plain<T>(c->M), nullptr, XINV_RHS, (const T*)c->M, out);
        if (st) return st;
        c->abm_slot = slot;
        c->abm_have_f = true;
        c->n_exact++;
    }
    const bool extrap = p >= 0 && (int)c->hist.size() == p;
    double h = s->h;
    if (s->adaptive) {
        if (c->h_next > 0) h = c->h_next;
        h = std::min(std::max(h, s->h_min), s->h_max);
    }
    int rejected = 0;
    bool forced = false;
    double err = -1.0, h_next = h;
    for (;;) {
        const bool prev = c->abm_have_prev;
        const double r = prev ? h / c->abm_hprev : 0.0;
        Combo<T> pr{};
        pr.base = (const T*)c->M;
        pr.f[0] = (const T*)c->F[0];
        pr.coef[0] = (T)(prev ? h * (1.0 + 0.5 * r) : h);
        pr.nf = 1;
        if (prev) {
            pr.f[1] = (const T*)c->F[2];
            pr.coef[1] = (T)(-0.5 * h * r);
            pr.nf = 2;
        }
        {
            PROF(LLGX_K_COMBINE);
            HIPCHK(c, launch_combine<T>(c->stream, 3 * c->ncell * c->nb, pr, (T*)c->Mk));
        }
        if (extrap) {
            Extrap<T> ex{};
            ex.n = 1;
            ex.w[0] = T(1);
            if (p == 0) {
                ex.g[0] = (const T*)c->G[c->abm_slot];
            } else {
                std::vector<double> nodes;
                EPoly<T> ep{};
                ep.ng = p + 1;
                ep.nd = 1;
                for (int i = 0; i < p; ++i) {
                    nodes.push_back(c->hist[i].t - c->t);
                    ep.g[i] = (const T*)c->G[c->hist[i].slot];
                }
                nodes.push_back(0.0);
                ep.g[p] = (const T*)c->G[c->abm_slot];
                const std::vector<double> w = lagrange(nodes, h);
                for (int i = 0; i <= p; ++i) ep.w[0][i] = (T)w[i];
                ep.out[0] = (T*)c->E[0];
                {
                    PROF(LLGX_K_EPOLY);
                    HIPCHK(c, launch_epoly<T>(c->stream, 3 * c->ncell * c->nb, ep));
                }
                ex.g[0] = (const T*)c->E[0];
            }
            PROF(LLGX_K_EXTRAP);
            HIPCHK(c, launch_extrap_rhs<T>(c->stream, plain<T>(c->Mk), ex, phys<T>(c), (T*)c->F[1],
                                           NextStage<T>{nullptr, nullptr, T(0)}));
            c->n_extrap++;
        } else {
            XinvOut out{nullptr, c->F[1], nullptr, nullptr, 0.0};
            llgx_status st = eval_exact<T>(c, plain<T>(c->Mk), nullptr, XINV_RHS, (const T*)c->Mk, out);
            if (st) return st;
            c->n_exact++;
        }
        // corrector and M_{n+1} - M_p = h (-(1+r)/2 F_n + F_p/2 + (r/2) F_{n-1})
        Final<T> fs{};
        fs.err = s->adaptive ? 1 : 0;
        const double k = prev ? r / (3.0 * (r + 1.0)) : 1.0;
        fs.f[0] = (const T*)c->F[0];
        fs.cb[0] = (T)(0.5 * h);
        fs.ce[0] = k * h * (prev ? -0.5 * (1.0 + r) : -0.5);
        fs.f[1] = (const T*)c->F[1];
        fs.cb[1] = (T)(0.5 * h);
        fs.ce[1] = k * h * 0.5;
        fs.n = 2;
        if (prev) {
            fs.f[2] = (const T*)c->F[2];
            fs.cb[2] = T(0);
            fs.ce[2] = k * h * 0.5 * r;
            fs.n = 3;
        }
        {
            PROF(LLGX_K_FINAL);
            HIPCHK(c, launch_final<T>(c->stream, c->ncell, c->nb, (const T*)c->M, fs, 1.0 / c->p.Ms, (T*)c->Mnew,
                                      c->parts, c->nparts));
        }
        if (!s->adaptive) break;
        {
            PROF(LLGX_K_OTHER);
            HIPCHK(c, launch_reduce_max(c->stream, c->parts, c->nparts, c->scal));
        }
        HIPCHK(c, hipMemcpyAsync(&err, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (!std::isfinite(err)) return c->fail(LLGX_E_NONFINITE, "non-finite error estimate at t=%g", c->t);
        const double cf =
            err <= 0.0 ? s->c_max : std::min(std::max(std::pow(0.8 * s->e_max / err, 1.0 / 3.0), s->c_min), s->c_max);
        if (err > s->e_max) {
            if (h > s->h_min) {
                rejected++;
                h = std::min(std::max(h * cf, s->h_min), s->h_max);
                continue;
            }
            forced = true;
        }
        h_next = std::min(std::max(h * cf, s->h_min), s->h_max);
        break;
    }
    // accept; F[0] still holds F_n at (t_n, M_n)
    double dmdt = -1.0;
    if (s->report_dmdt && info) {
        llgx_status st = read_max_dmdt<T>(c, &dmdt);
        if (st) return st;
    }
    if (p > 0) {
        c->hist.push_back({c->t, c->abm_slot});
        while ((int)c->hist.size() > p) c->hist.erase(c->hist.begin());
    }
    std::swap(c->M, c->Mnew);
    c->t += h;
    c->n_acc++;
    if (s->renormalize) {
        PROF(LLGX_K_OTHER);
        HIPCHK(c, launch_renorm<T>(c->stream, c->ncell, c->nb, (T*)c->M, c->p.Ms));
    }
    std::swap(c->F[2], c->F[0]);
    c->abm_hprev = h;
    c->abm_have_prev = true;
    const int slot = free_slot(c);
    XinvOut out{nullptr, c->F[0], p >= 0 ? c->G[slot] : nullptr, nullptr, 0.0};
    llgx_status st = eval_exact<T>(c, plain<T>(c->M), nullptr, XINV_RHS, (const T*)c->M, out);
    if (st) return st;
    c->abm_slot = slot;
    c->n_exact++;
    c->h_next = s->adaptive ? h_next : h;
    c->n_rej += rejected;
    c->n_forced += forced;
    if (info) {
        info->t = c->t;
        info->h_used = h;
        info->h_next = c->h_next;
        info->err = err;
        info->rejected = rejected;
        info->exact_evals = (int)(c->n_exact - ex0);
        info->extrap_evals = (int)(c->n_extrap - xt0);
        info->forced = forced;
        info->max_dmdt = dmdt;
    }
    return LLGX_OK;
}

template <typename T>
static llgx_status do_step(Ctx* c, const llgx_stepper* s, llgx_step_info* info) {
    const Tableau* tab;
    int p;
    llgx_status st = check_stepper(c, s, &tab, &p);
    if (st) return st;
    if (tab->multistep) return do_step_abm<T>(c, s, p, info);
    Plan pl{};
    pl.tab = tab;
    pl.p = p;
    pl.extrap = p >= 0 && (int)c->hist.size() == p;
    pl.stage1 = !c->fsal_valid;
    pl.slot0 = free_slot(c);
    pl.want_err = s->adaptive != 0;
    pl.in_place = s->adaptive == 0;  // a rejected attempt restarts from M0
    double h = s->h;
    if (s->adaptive) {
        if (c->h_next > 0) h = c->h_next;
        h = std::min(std::max(h, s->h_min), s->h_max);
    }
    const int q = s->exponent_mode == 1 ? tab->order : std::min(tab->order, tab->order_hat > 0 ? tab->order_hat : tab->order);
    const long long ex0 = c->n_exact, xt0 = c->n_extrap;
    int rejected = 0;
    bool forced = false;
    double err = -1.0, h_next = h;
    for (;;) {
        pl.h = h;
        st = enqueue_attempt<T>(c, pl);
        if (st) return st;
        if (pl.stage1) c->n_exact++;
        const int later = tab->S - 1;
        if (pl.extrap)
            c->n_extrap += later;
        else
            c->n_exact += later;
        if (!s->adaptive) break;
        HIPCHK(c, hipMemcpyAsync(&err, c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (!std::isfinite(err)) return c->fail(LLGX_E_NONFINITE, "non-finite error estimate at t=%g", c->t);
        const double cf =
            err <= 0.0 ? s->c_max
                       : std::min(std::max(std::pow(0.8 * s->e_max / err, 1.0 / (q + 1)), s->c_min), s->c_max);
        if (err > s->e_max) {
            if (h > s->h_min) {
                rejected++;
                h = std::min(std::max(h * cf, s->h_min), s->h_max);
                pl.stage1 = false;  // stage 1 does not depend on h: reuse it
                continue;
            }
            forced = true;
        }
        h_next = std::min(std::max(h * cf, s->h_min), s->h_max);
        break;
    }
    // F[0] holds the first stage's derivative at (t, M0) until commit
    double dmdt = -1.0;
    if (s->report_dmdt && info) {
        st = read_max_dmdt<T>(c, &dmdt);
        if (st) return st;
    }
    st = commit<T>(c, pl, h);
    if (st) return st;
    if (s->renormalize) {
        PROF(LLGX_K_OTHER);
        HIPCHK(c, launch_renorm<T>(c->stream, c->ncell, c->nb, (T*)c->M, c->p.Ms));
    }
    c->h_next = s->adaptive ? h_next : h;
    c->n_rej += rejected;
    c->n_forced += forced;
    if (info) {
        info->t = c->t;
        info->h_used = h;
        info->h_next = c->h_next;
        info->err = err;
        info->rejected = rejected;
        info->exact_evals = (int)(c->n_exact - ex0);
        info->extrap_evals = (int)(c->n_extrap - xt0);
        info->forced = forced;
        info->max_dmdt = dmdt;
    }
    return LLGX_OK;
}

// Fixed steps replayed from graphs capture up to this many consecutive
// steps in one graph: each graph launch costs the device several µs on its
// own (measured about 7 µs per launch of a chain of small kernels), which
// one step's graph would pay once per step.
constexpr int GRAPH_BLOCK_STEPS = 8;

// the plan of a graph-replayed fixed step from the handle's current state
static Plan fixed_plan(const Ctx* c, const Tableau* tab, int p, double h) {
    Plan pl{};
    pl.tab = tab;
    pl.p = p;
    pl.extrap = p >= 0;
    pl.stage1 = true;
    pl.slot0 = free_slot(c);
    pl.want_err = false;
    pl.in_place = true;
    pl.h = h;
    return pl;
}

// the host-side stepping state a step's commit changes
struct StepState {
    std::vector<Ctx::Hist> hist;
    void* M;
    void* Mnew;
    void* F[MAX_F];
    bool fsal_valid;
    double t;
    long long n_acc;
    explicit StepState(const Ctx* c)
        : hist(c->hist), M(c->M), Mnew(c->Mnew), fsal_valid(c->fsal_valid), t(c->t), n_acc(c->n_acc) {
        std::copy(c->F, c->F + MAX_F, F);
    }
    void restore(Ctx* c) const {
        c->hist = hist;
        c->M = M;
        c->Mnew = Mnew;
        std::copy(F, F + MAX_F, c->F);
        c->fsal_valid = fsal_valid;
        c->t = t;
        c->n_acc = n_acc;
    }
};

template <typename T>
static llgx_status do_run_fixed(Ctx* c, const llgx_stepper* s, int64_t nsteps, int use_graph, llgx_step_info* info) {
    if (s && s->adaptive) return c->fail(LLGX_E_ARG, "llgx_run_fixed needs a fixed step (adaptive = 0)");
    // no per-step synchronisation: the |dM/dt| diagnostic is not reported
    llgx_stepper sf{};
    if (s) {
        sf = *s;
        sf.report_dmdt = 0;
        s = &sf;
    }
    int64_t i = 0;
    while (i < nsteps) {
        const Tableau* tab;
        int p;
        llgx_status st = check_stepper(c, s, &tab, &p);
        if (st) return st;
        const bool steady = !tab->multistep && ((p < 0 && !tab->fsal) || (p >= 0 && (int)c->hist.size() == p) ||
                                                (p < 0 && tab->fsal && s->renormalize));
        // the Lagrange nodes are relative times: graphs are reused only while steps stay uniform
        bool uniform = true;
        for (size_t j = 0; j < c->hist.size(); ++j) {
            const double expect = -(double)(c->hist.size() - j) * s->h;
            if (std::fabs((c->hist[j].t - c->t) - expect) > 1e-9 * s->h) uniform = false;
        }
        // the legacy default stream cannot be captured: replay needs a created stream
        if (!use_graph || !steady || !uniform || c->stream == nullptr || c->prof) {
            st = do_step<T>(c, s, info);
            if (st) return st;
            ++i;
            continue;
        }
        // a steady, uniform step is followed by steady, uniform steps: the
        // next `nb` steps are one graph
        const int nb = nsteps - i >= GRAPH_BLOCK_STEPS ? GRAPH_BLOCK_STEPS : 1;
        GraphKey key{c->M, free_slot(c), {}, s->h, s->method, p, c->kernel_gen, nb};
        for (auto& hh : c->hist) key.hist_slots.push_back(hh.slot);
        auto it = c->graphs.find(key);
        if (it == c->graphs.end()) {
            // capture the steps' launches (Eq. (3)-(6) attempts, renormalisation)
            // on a copy of the stepping state, restored afterwards
            const StepState saved(c);
            hipGraph_t g;
            HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            hipError_t e = hipSuccess;
            for (int k = 0; k < nb && st == LLGX_OK && e == hipSuccess; ++k) {
                const Plan pl = fixed_plan(c, tab, p, s->h);
                st = enqueue_attempt<T>(c, pl);
                if (st == LLGX_OK) st = commit<T>(c, pl, s->h);
                if (st == LLGX_OK && s->renormalize) e = launch_renorm<T>(c->stream, c->ncell, c->nb, (T*)c->M, c->p.Ms);
            }
            hipError_t e2 = hipStreamEndCapture(c->stream, &g);
            saved.restore(c);
            if (st) {
                if (e2 == hipSuccess) (void)hipGraphDestroy(g);
                return st;
            }
            if (e != hipSuccess || e2 != hipSuccess) {
                if (e2 == hipSuccess) (void)hipGraphDestroy(g);
                return c->fail(LLGX_E_HIP, "graph capture failed: %s", hipGetErrorString(e != hipSuccess ? e : e2));
            }
            hipGraphExec_t ge;
            e = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
            (void)hipGraphDestroy(g);
            if (e != hipSuccess) return c->fail(LLGX_E_HIP, "graph instantiation failed: %s", hipGetErrorString(e));
            it = c->graphs.emplace(key, ge).first;
        }
        HIPCHK(c, hipGraphLaunch(it->second, c->stream));
        // the host side of the replayed steps
        for (int k = 0; k < nb; ++k) {
            const Plan pl = fixed_plan(c, tab, p, s->h);
            c->n_exact += 1 + (pl.extrap ? 0 : tab->S - 1);
            c->n_extrap += pl.extrap ? tab->S - 1 : 0;
            st = commit<T>(c, pl, s->h);
            if (st) return st;
        }
        c->h_next = s->h;
        if (info) {
            info->t = c->t;
            info->h_used = s->h;
            info->h_next = s->h;
            info->err = -1.0;
            info->rejected = 0;
            info->exact_evals = 1 + (p >= 0 ? 0 : tab->S - 1);
            info->extrap_evals = p >= 0 ? tab->S - 1 : 0;
            info->forced = 0;
            info->max_dmdt = -1.0;
        }
        i += nb;
    }
    return LLGX_OK;
}

template <typename T>
static llgx_status mean_m(Ctx* c, double out[3]) {
    HIPCHK(c, launch_mean<T>(c->stream, c->ncell, (const T*)c->M, c->parts, c->nparts));
    HIPCHK(c, launch_reduce_sum3(c->stream, c->parts, c->nparts, c->scal + 1));
    HIPCHK(c, hipMemcpyAsync(out, c->scal + 1, 3 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int i = 0; i < 3; ++i) out[i] /= (double)c->ncell;
    return LLGX_OK;
}

template <typename T>
static llgx_status do_run(Ctx* c, const llgx_stepper* s, double t_end, double sample_dt, double* mavg, int64_t cap,
                          int64_t* nsamples) {
    int64_t ns = 0;
    auto record = [&]() -> llgx_status {
        if (!mavg || ns >= cap) return LLGX_OK;
        llgx_status st = mean_m<T>(c, mavg + 3 * ns);
        if (st) return st;
        ns++;
        return LLGX_OK;
    };
    llgx_stepper sc = *s;
    sc.report_dmdt = 0;  // steps report nothing to the caller here
    llgx_status st = LLGX_OK;
    double next_s = 0.0;
    if (sample_dt > 0) {
        st = record();
        if (st) return st;
        next_s = c->t + sample_dt;
    }
    const double tol = 1e-9 * s->h;
    while (c->t < t_end - tol) {
        const Tableau* tab;
        int p;
        st = check_stepper(c, &sc, &tab, &p);
        if (st) return st;
        const double target = sample_dt > 0 ? std::min(next_s, t_end) : t_end;
        bool shortened = false;
        double h_prop = c->h_next > 0 ? c->h_next : sc.h;
        if (sc.adaptive && c->t + h_prop > target) {
            c->h_next = target - c->t;
            shortened = true;
        }
        llgx_step_info info;
        st = do_step<T>(c, &sc, &info);
        if (st) return st;
        if (shortened) c->h_next = std::max(c->h_next, h_prop);
        if (sample_dt > 0 && c->t >= next_s - 1e-9 * info.h_used) {
            st = record();
            if (st) return st;
            next_s += sample_dt;
        }
    }
    if (nsamples) *nsamples = ns;
    return LLGX_OK;
}

static void release(Ctx* c) {
    for (auto& m : c->marks) {
        (void)hipEventDestroy(m.a);
        (void)hipEventDestroy(m.b);
    }
    for (auto e : c->spare) (void)hipEventDestroy(e);
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    void* ptrs[] = {c->kfold, c->specA, c->specB,  c->M,      c->Mnew, c->Mk,
                    c->mk2_in_b ? nullptr : c->Mk2, c->parts, c->scal, c->octant, c->hab, c->empty_flag};
    for (void* p : ptrs)
        if (p) (void)hipFree(p);
    for (int i = 0; i < MAX_F; ++i)
        if (c->F[i]) (void)hipFree(c->F[i]);
    for (int i = 0; i < MAX_HIST; ++i)
        if (c->G[i]) (void)hipFree(c->G[i]);
    for (int i = 0; i < MAX_F; ++i)
        if (c->E[i] && !c->e_in_b[i]) (void)hipFree(c->E[i]);
    for (auto& kv : c->tw_work) (void)hipFree(kv.second);
    for (auto& kv : c->tw_f64) (void)hipFree(kv.second);
}

}  // namespace llgx

using namespace llgx;

// ===========================================================================
// C ABI

extern "C" {

const char* llgx_last_error(llgx_handle h) {
    if (!h) return g_create_error.c_str();
    return ((Ctx*)h)->err.c_str();
}

void llgx_stepper_defaults(llgx_stepper* s) {
    if (!s) return;
    std::memset(s, 0, sizeof *s);
    s->method = LLGX_RK4;
    s->extrap = LLGX_EXTRAP_FULL;
    s->adaptive = 0;
    s->renormalize = 0;
    s->exponent_mode = 0;
    s->h = 1e-13;
    s->h_min = 1e-15;
    s->h_max = 3e-12;
    s->c_min = 0.01;
    s->c_max = 2.0;
    s->e_max = 1e-5;
}

}  // extern "C"

namespace llgx {

// Context for nb samples of one problem (differing only in the applied field,
// ha_list[nb][3], or all equal to p->Ha when ha_list is null).
// ---- autotuner ----------------------------------------------------------
// Each FFT pass has launch variants (tile widths, rows per workgroup) with
// bit-identical results.  llgx_autotune times every variant of every pass on
// the handle's own shapes and keeps the fastest; the choice is remembered per
// (precision, spectral storage, mesh, samples) for the rest of the process
// and can be exported / imported as JSON lines.
static const int kNumVar[5] = {NVAR_XFWD, NVAR_COL, NVAR_ZMUL, NVAR_COL, NVAR_XINV};
constexpr int kMaxVar = 8;      // bound of every NVAR_*
constexpr int kTuneRounds = 3;  // interleaved timing rounds of the autotuner
static_assert(NVAR_XFWD <= kMaxVar && NVAR_COL <= kMaxVar && NVAR_ZMUL <= kMaxVar && NVAR_XINV <= kMaxVar,
              "launch variant count above kMaxVar");

struct TuneEntry {
    int var[5];
    double us[5];
};
static std::mutex g_tune_mu;
static std::map<std::string, TuneEntry> g_tune;

static std::string tune_key(const Ctx* c) {
    char b[160];
    snprintf(b, sizeof b, "%s/%s/%dx%dx%d/%d", c->prec == LLGX_F32 ? "f32" : "f64",
             c->spectral == LLGX_SPEC_BF16 ? "bf16" : c->spectral == LLGX_SPEC_F16 ? "f16" : "native", c->nx, c->ny,
             c->nz, c->nb);
    return b;
}

static void drop_graphs(Ctx* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
}

static void apply_tuned(Ctx* c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tune.find(tune_key(c));
    if (it == g_tune.end()) return;
    for (int k = 0; k < 5; ++k) c->var[k] = it->second.var[k];
    drop_graphs(c);
}

static llgx_status time_pass_any(Ctx* c, int kind, int v, int reps, double* us) {
    if (c->prec == LLGX_F64) return time_pass<double, double>(c, kind, v, reps, us);
    if (c->spectral == LLGX_SPEC_BF16) return time_pass<float, __bf16>(c, kind, v, reps, us);
    if (c->spectral == LLGX_SPEC_F16) return time_pass<float, _Float16>(c, kind, v, reps, us);
    return time_pass<float, float>(c, kind, v, reps, us);
}

static llgx_status tune_ctx(Ctx* c, int reps, double us_out[5]) {
    if (reps < 1) return c->fail(LLGX_E_ARG, "reps must be >= 1");
    if (!c->have_kernel) return c->fail(LLGX_E_STATE, "demag kernel not computed (llgx_precompute_demag)");
    if (!c->have_m) return c->fail(LLGX_E_STATE, "magnetization not set (llgx_set_m)");
    TuneEntry te{};
    for (int k = 0; k < 5; ++k) {
        te.var[k] = 0;
        te.us[k] = 0.0;
        if (!pass_exists(c, k)) continue;
        // the variants take turns over kTuneRounds rounds and each keeps its
        // fastest round, so a clock ramp or a burst of other work during one
        // variant's measurement does not decide the choice
        double t[kMaxVar];
        for (int v = 0; v < kNumVar[k]; ++v) t[v] = 0.0;
        for (int r = 0; r < kTuneRounds; ++r) {
            for (int v = 0; v < kNumVar[k]; ++v) {
                double us = 0.0;
                llgx_status st = time_pass_any(c, k, v, reps, &us);
                if (st) return st;
                if (r == 0 || us < t[v]) t[v] = us;
            }
        }
        for (int v = 0; v < kNumVar[k]; ++v) {
            if (v == 0 || t[v] < te.us[k]) {
                te.us[k] = t[v];
                te.var[k] = v;
            }
        }
    }
    for (int k = 0; k < 5; ++k) {
        c->var[k] = te.var[k];
        if (us_out) us_out[k] = te.us[k];
    }
    drop_graphs(c);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(c)] = te;
    return LLGX_OK;
}

// Device address of this device's `scratch`, resolved once per device with
// that device current (the one the handle is created on).
static llgx_status scratch_address(Ctx* c) {
    int dev = -1;
    HIPCHK(c, hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    auto it = g_scratch_dev.find(dev);
    if (it == g_scratch_dev.end()) {
        void* ptr = nullptr;
        HIPCHK(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        if (!ptr) return c->fail(LLGX_E_HIP, "hipGetSymbolAddress gave no address for the scratch array");
        it = g_scratch_dev.emplace(dev, ptr).first;
    }
    c->noalloc = it->second;
    return LLGX_OK;
}

static llgx_status create_ctx(const llgx_problem* p, int nb, const double* ha_list, int32_t precision,
                              int32_t spectral, void* hip_stream, Ctx** out, std::string& err) {
    *out = nullptr;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1 || !(p->dx > 0) || !(p->dy > 0) || !(p->dz > 0) || !(p->Ms > 0) ||
        !(p->gamma > 0) || p->A < 0 || p->alpha < 0) {
        err = "invalid problem (sizes >= 1, cell > 0, Ms > 0, gamma > 0, A >= 0, alpha >= 0)";
        return LLGX_E_ARG;
    }
    if (precision != LLGX_F32 && precision != LLGX_F64) {
        err = "precision must be LLGX_F32 or LLGX_F64";
        return LLGX_E_ARG;
    }
    if (spectral != LLGX_SPEC_NATIVE && spectral != LLGX_SPEC_BF16 && spectral != LLGX_SPEC_F16) {
        err = "spectral must be LLGX_SPEC_NATIVE, LLGX_SPEC_BF16 or LLGX_SPEC_F16";
        return LLGX_E_ARG;
    }
    if (spectral != LLGX_SPEC_NATIVE && precision != LLGX_F32) {
        err = "16-bit spectral storage requires LLGX_F32";
        return LLGX_E_ARG;
    }
    Ctx* c = new Ctx();
    c->p = *p;
    c->prec = precision;
    c->spectral = spectral;
    c->stream = (hipStream_t)hip_stream;
    c->tsz = precision == LLGX_F32 ? 4 : 8;
    c->nx = p->nx;
    c->ny = p->ny;
    c->nz = p->nz;
    c->nb = nb;
    c->ncell = (long)p->nx * p->ny * p->nz;
    c->Px = p->nx > 1 ? next_pow2(2L * p->nx - 1) : 1;
    c->Py = p->ny > 1 ? next_pow2(2L * p->ny - 1) : 1;
    c->Pz = p->nz > 1 ? next_pow2(2L * p->nz - 1) : 1;
    if (c->Px > MAX_LEN || c->Py > MAX_LEN || c->Pz > MAX_LEN / 2) {
        err = "mesh too large: padded FFT length above 2048 (x, y) or 1024 (z)";
        delete c;
        return LLGX_E_UNSUPPORTED;
    }
    c->LX = c->Px > 1 ? c->Px / 2 : 0;
    c->Kx = c->Px > 1 ? c->Px / 2 + 1 : 1;
    c->SX = (c->Kx + 15) / 16 * 16;
    c->Kyf = c->Py > 1 ? c->Py / 2 + 1 : 1;
    c->Kzf = c->Pz > 1 ? c->Pz / 2 + 1 : 1;
    const size_t cbytes = spectral == LLGX_SPEC_NATIVE ? 2 * c->tsz : 4;  // bytes per stored complex value
    const size_t vbytes = 3 * (size_t)c->ncell * nb * c->tsz;
    llgx_status st = LLGX_OK;
    auto A = [&](void** ptr, size_t bytes) {
        if (st == LLGX_OK) st = dalloc(c, ptr, bytes);
    };
    const size_t bytesA = 3 * (size_t)c->nz * c->ny * c->SX * cbytes * nb;
    const size_t bytesB = 3 * (size_t)c->nz * c->Py * c->SX * cbytes * nb;
    A(&c->specA, bytesA);
    if (c->Py > 1) A(&c->specB, bytesB);
    A(&c->M, vbytes);
    A(&c->Mnew, vbytes);
    A(&c->Mk, vbytes);
    for (int i = 0; i < MAX_F; ++i) A(&c->F[i], vbytes);
    for (int i = 0; i < MAX_HIST; ++i) A(&c->G[i], vbytes);
    // The second stage-input buffer and the Eq. (6) fields are live only
    // between the stage-1 evaluation of an extrapolated attempt and its
    // Eq. (3) update, when spectrum B (used only inside an exact evaluation)
    // is dead: they are placed inside B while it has room.  One step then
    // touches less memory (at the benchmark mesh 229 instead of 279 MB),
    // which stays inside the 256 MB Infinity Cache in front of HBM.  B is
    // rewritten in full by every y forward pass before it is read (its
    // padding columns past Kx are never read), so what these buffers leave
    // in it does not matter.
    const size_t vslot = (vbytes + 255) / 256 * 256;
    size_t bused = 0;
    if (st == LLGX_OK && c->specB && bytesB >= vslot) {
        c->Mk2 = c->specB;
        c->mk2_in_b = true;
        bused = vslot;
    } else {
        A(&c->Mk2, vbytes);
    }
    for (int i = 0; i < MAX_F - 1; ++i) {
        if (st == LLGX_OK && c->specB && bused + vslot <= bytesB) {
            c->E[i] = (char*)c->specB + bused;
            c->e_in_b[i] = true;
            bused += vslot;
        } else {
            A(&c->E[i], vbytes);
        }
    }
    c->nparts = (int)std::min<long>(1024, std::max<long>(1, (c->ncell * nb + 255) / 256));
    c->nparts_alloc = std::max<long>(c->nparts, cell_grid(c->nx, c->ny, c->nz, nb).nblocks);
    A((void**)&c->parts, 3 * (size_t)c->nparts_alloc * sizeof(double));
    A((void**)&c->scal, 8 * sizeof(double));
    A((void**)&c->empty_flag, 16);
    A(&c->hab, 3 * (size_t)nb * c->tsz);
    if (st == LLGX_OK) {
        // padding columns of the spectra are read (never used) by 16-byte packs: keep them zero
        if (hipMemset(c->specA, 0, bytesA) != hipSuccess) st = c->fail(LLGX_E_HIP, "hipMemset failed");
        if (st == LLGX_OK && c->specB && hipMemset(c->specB, 0, bytesB) != hipSuccess)
            st = c->fail(LLGX_E_HIP, "hipMemset failed");
        if (st == LLGX_OK && hipMemset(c->empty_flag, 0, 16) != hipSuccess) st = c->fail(LLGX_E_HIP, "hipMemset failed");
    }
    if (st == LLGX_OK) {
        // each sample's applied field (the problem's own when no list is given)
        std::vector<char> hb(3 * (size_t)nb * c->tsz);
        for (int i = 0; i < 3 * nb; ++i) {
            const double v = ha_list ? ha_list[i] : c->p.Ha[i % 3];
            if (c->tsz == 4)
                ((float*)hb.data())[i] = (float)v;
            else
                ((double*)hb.data())[i] = v;
        }
        if (hipMemcpy(c->hab, hb.data(), hb.size(), hipMemcpyHostToDevice) != hipSuccess)
            st = c->fail(LLGX_E_HIP, "hipMemcpy of applied fields failed");
    }
    if (st == LLGX_OK) {
        for (int L : {c->LX, c->Px, c->Py, c->Pz}) {
            if (st) break;
            st = c->prec == LLGX_F32 ? make_table<float>(c, c->tw_work, L) : make_table<double>(c, c->tw_work, L);
        }
    }
    if (st != LLGX_OK) {
        err = c->err;
        release(c);
        delete c;
        return st;
    }
    if (st == LLGX_OK) st = scratch_address(c);
    if (st != LLGX_OK) {
        err = c->err;
        release(c);
        delete c;
        return st;
    }
    apply_tuned(c);
    *out = c;
    return LLGX_OK;
}

// Independent samples grouped by problem (all fields but the applied one):
// each group is one context whose launches cover all its samples.
struct Batch {
    std::vector<Ctx*> groups;
    std::vector<std::pair<int, int>> where;  // sample -> (group, index in group)
    hipStream_t stream = nullptr;
    std::string err;
    std::map<std::vector<GraphKey>, hipGraphExec_t> graphs;
    // groups 1.. get streams of their own (default priority) inside a captured
    // step, forked from and joined back into `stream`, so meshes of different
    // shapes run side by side
    std::vector<hipStream_t> gstreams;
    std::vector<hipEvent_t> joins;
    hipEvent_t fork = nullptr;
    // LLGX_BATCH_STREAMS (default): the groups' own launches on forked
    // streams; LLGX_BATCH_JOBS: each pass of a captured step is one
    // launch over a job table of the mesh groups (per FFT length
    // for the FFT passes; up to BMAX groups a launch), where every launch of
    // the step has that form (else the forked-stream capture)
    int mode = LLGX_BATCH_STREAMS;
    std::vector<void*> tables;  // device job tables of the captured job-table steps
    std::vector<hipEvent_t> cap_events;  // fork/join events of the captured job-table steps
    int last_jobs = 0, last_kernels = 0;
};

// the streams and events of forked captures: ng - 1 side streams (default
// priority) and their join events, and the fork event
static llgx_status fork_streams(Batch* bt, size_t ng) {
    if (ng < 2 || !bt->gstreams.empty()) return LLGX_OK;
    hipError_t e = hipEventCreateWithFlags(&bt->fork, hipEventDisableTiming);
    for (size_t g = 1; g < ng && e == hipSuccess; ++g) {
        hipStream_t gs = nullptr;
        hipEvent_t je = nullptr;
        e = hipStreamCreateWithFlags(&gs, hipStreamNonBlocking);
        if (e == hipSuccess) bt->gstreams.push_back(gs);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&je, hipEventDisableTiming);
        if (e == hipSuccess) bt->joins.push_back(je);
    }
    if (e != hipSuccess) {
        bt->err = "stream creation failed";
        return LLGX_E_HIP;
    }
    return LLGX_OK;
}

static bool same_material(const llgx_problem& a, const llgx_problem& b) {
    return a.nx == b.nx && a.ny == b.ny && a.nz == b.nz && a.dx == b.dx && a.dy == b.dy && a.dz == b.dz &&
           a.Ms == b.Ms && a.A == b.A && a.K == b.K && a.easy[0] == b.easy[0] && a.easy[1] == b.easy[1] &&
           a.easy[2] == b.easy[2] && a.alpha == b.alpha && a.gamma == b.gamma;
}

// Capture one step of every group as job-table launches: each group's
// launches are recorded (enqueue_attempt with Ctx::rec), the i-th launches
// of all groups are joined into one job table per FFT length and BMAX
// groups (a group without the pass, a one-row mesh's y passes, takes no
// part), the tables are copied to device memory (kept for the graph's
// lifetime), and the launches are captured on the batch stream, those of
// one pass side by side on forked streams.  LLGX_E_UNSUPPORTED (nothing
// captured) when some launch has no job-table form or the groups' launch
// sequences differ (then the forked-stream capture is used).
template <typename T>
static llgx_status capture_jobs(Batch* bt, const std::vector<Plan>& plans, hipGraphExec_t* out, int* nkern) {
    const size_t ng = bt->groups.size();
    std::vector<std::vector<Ctx::Rec>> recs(ng);
    bool ok = true;
    for (size_t g = 0; g < ng; ++g) {
        Ctx* c = bt->groups[g];
        c->rec = &recs[g];
        c->rec_unsupported = false;
        llgx_status st = enqueue_attempt<T>(c, plans[g]);
        c->rec = nullptr;
        if (st) {
            bt->err = c->err;
            return st;
        }
        ok = ok && !c->rec_unsupported && recs[g].size() == recs[0].size();
        for (size_t i = 0; ok && i < recs[g].size(); ++i)
            ok = recs[g][i].kind == recs[0][i].kind && recs[g][i].nf == recs[0][i].nf;
    }
    if (!ok) {
        bt->err = "job-table launch not used: a launch without job-table form, or groups with different launches";
        return LLGX_E_UNSUPPORTED;
    }
    std::vector<unsigned char> blob;
    // launches of the i-th recorded launch: one per FFT length (and BMAX
    // groups), independent of each other
    std::vector<std::vector<BatchLaunch>> levels(recs[0].size());
    size_t width = 1, nlaunch = 0;
    for (size_t i = 0; i < recs[0].size(); ++i) {
        // the groups of each FFT length (one key for the per-cell kinds)
        std::map<int, std::vector<const void*>> by_len;
        for (size_t g = 0; g < ng; ++g) {
            const int key = batch_instance<T>(recs[0][i].kind, recs[g][i].arg.data());
            if (key >= 0) by_len[key].push_back(recs[g][i].arg.data());
        }
        for (auto& kv : by_len) {
            for (size_t g0 = 0; g0 < kv.second.size(); g0 += BMAX) {
                std::vector<const void*> args(kv.second.begin() + g0,
                                              kv.second.begin() + std::min(kv.second.size(), g0 + BMAX));
                BatchLaunch bl{};
                hipError_t e = prepare_batch<T>(recs[0][i].kind, recs[0][i].nf, args, blob, bl);
                if (e == hipErrorInvalidValue) {
                    bt->err = "job-table launch not used: launch " + std::to_string(i) + " (kind " +
                              std::to_string(recs[0][i].kind) + ") outside the job-table kernels' lengths";
                    return LLGX_E_UNSUPPORTED;
                }
                if (e != hipSuccess) {
                    bt->err = std::string("job-table launch setup failed: ") + hipGetErrorString(e);
                    return LLGX_E_HIP;
                }
                levels[i].push_back(bl);
            }
        }
        width = std::max(width, levels[i].size());
        nlaunch += levels[i].size();
    }
    if (llgx_status fs = fork_streams(bt, ng)) return fs;
    if (bt->gstreams.size() + 1 < width) {
        bt->err = "job-table launch not used: more launches of one pass than side streams";
        return LLGX_E_UNSUPPORTED;
    }
    void* dev = nullptr;
    if (hipMalloc(&dev, std::max<size_t>(blob.size(), 256)) != hipSuccess) {
        bt->err = "job table allocation failed";
        return LLGX_E_OOM;
    }
    bt->tables.push_back(dev);
    if (hipMemcpy(dev, blob.data(), blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
        bt->err = "job table copy failed";
        return LLGX_E_HIP;
    }
    hipGraph_t gr;
    if (hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        bt->err = "graph capture could not start";
        return LLGX_E_HIP;
    }
    // the launches of one level run side by side: launch 0 on the batch
    // stream, launch j on side stream j - 1, forked from and joined back into
    // the batch stream (events of their own, kept until the batch is
    // destroyed)
    hipError_t e = hipSuccess;
    auto event = [&](hipEvent_t* ev) {
        if (e == hipSuccess) e = hipEventCreateWithFlags(ev, hipEventDisableTiming);
        if (e == hipSuccess) bt->cap_events.push_back(*ev);
    };
    for (size_t i = 0; i < levels.size() && e == hipSuccess; ++i) {
        const std::vector<BatchLaunch>& lv = levels[i];
        if (lv.empty()) continue;
        hipEvent_t fk = nullptr;
        std::vector<hipEvent_t> jn(lv.size(), nullptr);
        if (lv.size() > 1) {
            event(&fk);
            if (e == hipSuccess) e = hipEventRecord(fk, bt->stream);
        }
        for (size_t j = 1; j < lv.size() && e == hipSuccess; ++j) {
            hipStream_t ss = bt->gstreams[j - 1];
            e = hipStreamWaitEvent(ss, fk, 0);
            if (e == hipSuccess) e = enqueue_batch(lv[j], (const char*)dev + lv[j].offset, ss);
            event(&jn[j]);
            if (e == hipSuccess) e = hipEventRecord(jn[j], ss);
        }
        if (e == hipSuccess) e = enqueue_batch(lv[0], (const char*)dev + lv[0].offset, bt->stream);
        for (size_t j = 1; j < lv.size() && e == hipSuccess; ++j) e = hipStreamWaitEvent(bt->stream, jn[j], 0);
    }
    hipError_t e2 = hipStreamEndCapture(bt->stream, &gr);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (e2 == hipSuccess) (void)hipGraphDestroy(gr);
        bt->err = std::string("job-table capture failed: ") + hipGetErrorString(e != hipSuccess ? e : e2);
        return LLGX_E_HIP;
    }
    hipGraphExec_t ge;
    e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
        bt->err = "graph instantiation failed";
        return LLGX_E_HIP;
    }
    *out = ge;
    *nkern = (int)nlaunch;
    return LLGX_OK;
}

// One accepted step of every sample with one h for all: each group runs its
// attempt (Eq. (3)-(6)), the error norm of the attempt is the maximum of the
// groups' norms (each the maximum over its samples' cells), and the Eq. (5)
// controller of Sec. II accepts or rejects the attempt for all samples
// together.  Each group keeps its own priming and history.
template <typename T>
static llgx_status batch_step(Batch* bt, const llgx_stepper* s, llgx_step_info* info) {
    if (!s) {
        bt->err = "null stepper";
        return LLGX_E_ARG;
    }
    const size_t ng = bt->groups.size();
    std::vector<Plan> plans(ng);
    const Tableau* tab = nullptr;
    for (size_t g = 0; g < ng; ++g) {
        Ctx* c = bt->groups[g];
        int p;
        llgx_status st = check_stepper(c, s, &tab, &p);
        if (st) {
            bt->err = c->err;
            return st;
        }
        if (tab->multistep) {
            bt->err = "ABM2 is stepped per handle, not in batches";
            return LLGX_E_UNSUPPORTED;
        }
        Plan& pl = plans[g];
        pl.tab = tab;
        pl.p = p;
        pl.extrap = p >= 0 && (int)c->hist.size() == p;
        pl.stage1 = !c->fsal_valid;
        pl.slot0 = free_slot(c);
        pl.want_err = s->adaptive != 0;
        pl.in_place = s->adaptive == 0;  // a rejected attempt restarts from M0
    }
    Ctx* c0 = bt->groups[0];
    double h = s->h;
    if (s->adaptive) {
        if (c0->h_next > 0) h = c0->h_next;
        h = std::min(std::max(h, s->h_min), s->h_max);
    }
    const int q = s->exponent_mode == 1 ? tab->order
                                        : std::min(tab->order, tab->order_hat > 0 ? tab->order_hat : tab->order);
    const long long ex0 = c0->n_exact, xt0 = c0->n_extrap;
    int rejected = 0;
    bool forced = false;
    double err = -1.0, h_next = h;
    std::vector<double> errs(ng, 0.0);
    for (;;) {
        for (size_t g = 0; g < ng; ++g) {
            Ctx* c = bt->groups[g];
            Plan& pl = plans[g];
            pl.h = h;
            llgx_status st = enqueue_attempt<T>(c, pl);
            if (st) {
                bt->err = c->err;
                return st;
            }
            if (pl.stage1) c->n_exact++;
            if (pl.extrap)
                c->n_extrap += tab->S - 1;
            else
                c->n_exact += tab->S - 1;
            if (s->adaptive &&
                hipMemcpyAsync(&errs[g], c->scal, sizeof(double), hipMemcpyDeviceToHost, c->stream) != hipSuccess) {
                bt->err = "error-norm copy failed";
                return LLGX_E_HIP;
            }
        }
        if (!s->adaptive) break;
        if (hipStreamSynchronize(bt->stream) != hipSuccess) {
            bt->err = "synchronisation failed";
            return LLGX_E_HIP;
        }
        err = 0.0;
        for (double e : errs) err = std::isfinite(e) && std::isfinite(err) ? std::max(err, e) : NAN;
        if (!std::isfinite(err)) {
            bt->err = "non-finite error estimate";
            return LLGX_E_NONFINITE;
        }
        const double cf =
            err <= 0.0 ? s->c_max
                       : std::min(std::max(std::pow(0.8 * s->e_max / err, 1.0 / (q + 1)), s->c_min), s->c_max);
        if (err > s->e_max) {
            if (h > s->h_min) {
                rejected++;
                h = std::min(std::max(h * cf, s->h_min), s->h_max);
                for (Plan& pl : plans) pl.stage1 = false;  // stage 1 does not depend on h: reuse it
                continue;
            }
            forced = true;
        }
        h_next = std::min(std::max(h * cf, s->h_min), s->h_max);
        break;
    }
    for (size_t g = 0; g < ng; ++g) {
        Ctx* c = bt->groups[g];
        llgx_status st = commit<T>(c, plans[g], h);
        if (st) {
            bt->err = c->err;
            return st;
        }
        if (s->renormalize && launch_renorm<T>(c->stream, c->ncell, c->nb, (T*)c->M, c->p.Ms) != hipSuccess) {
            bt->err = "renormalisation launch failed";
            return LLGX_E_HIP;
        }
        c->h_next = s->adaptive ? h_next : h;
        c->n_rej += rejected;
        c->n_forced += forced;
    }
    if (info) {
        info->t = c0->t;
        info->h_used = h;
        info->h_next = c0->h_next;
        info->err = err;
        info->rejected = rejected;
        info->exact_evals = (int)(c0->n_exact - ex0);
        info->extrap_evals = (int)(c0->n_extrap - xt0);
        info->forced = forced;
        info->max_dmdt = -1.0;
    }
    return LLGX_OK;
}

template <typename T>
static llgx_status batch_run_fixed(Batch* bt, const llgx_stepper* s, int64_t nsteps, int use_graph) {
    if (!s || s->adaptive) {
        bt->err = "batched runs take a fixed step (adaptive = 0)";
        return LLGX_E_ARG;
    }
    if (tableau_for(s->method) && tableau_for(s->method)->multistep) {
        bt->err = "ABM2 is stepped per handle, not in batches";
        return LLGX_E_UNSUPPORTED;
    }
    for (int64_t i = 0; i < nsteps; ++i) {
        bool steady = use_graph && bt->stream != nullptr;
        std::vector<Plan> plans(bt->groups.size());
        std::vector<GraphKey> keys;
        for (size_t g = 0; g < bt->groups.size(); ++g) {
            Ctx* c = bt->groups[g];
            const Tableau* tab;
            int p;
            llgx_status st = check_stepper(c, s, &tab, &p);
            if (st) {
                bt->err = c->err;
                return st;
            }
            const bool ok = ((p < 0 && !tab->fsal) || (p >= 0 && (int)c->hist.size() == p) ||
                             (p < 0 && tab->fsal && s->renormalize)) && !c->prof;
            for (size_t j = 0; j < c->hist.size(); ++j) {
                const double expect = -(double)(c->hist.size() - j) * s->h;
                if (std::fabs((c->hist[j].t - c->t) - expect) > 1e-9 * s->h) steady = false;
            }
            steady = steady && ok;
            Plan& pl = plans[g];
            pl.tab = tab;
            pl.p = p;
            pl.extrap = p >= 0;
            pl.stage1 = true;
            pl.slot0 = free_slot(c);
            pl.want_err = false;
            pl.in_place = true;
            pl.h = s->h;
            GraphKey key{c->M, pl.slot0, {}, s->h, s->method, p, c->kernel_gen};
            for (auto& hh : c->hist) key.hist_slots.push_back(hh.slot);
            keys.push_back(key);
        }
        if (!steady) {
            for (Ctx* c : bt->groups) {
                llgx_status st = do_step<T>(c, s, nullptr);
                if (st) {
                    bt->err = c->err;
                    return st;
                }
            }
            continue;
        }
        auto it = bt->graphs.find(keys);
        if (it == bt->graphs.end() && bt->mode == LLGX_BATCH_JOBS) {
            hipGraphExec_t ge;
            int nk = 0;
            llgx_status st = capture_jobs<T>(bt, plans, &ge, &nk);
            if (st == LLGX_OK) {
                it = bt->graphs.emplace(keys, ge).first;
                bt->last_jobs = 1;
                bt->last_kernels = nk;
            } else if (st != LLGX_E_UNSUPPORTED) {
                return st;
            }
        }
        if (it == bt->graphs.end()) {
            hipGraph_t gr;
            if (hipStreamBeginCapture(bt->stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
                bt->err = "graph capture could not start";
                return LLGX_E_HIP;
            }
            const size_t ng = bt->groups.size();
            llgx_status st = fork_streams(bt, ng);
            if (st == LLGX_OK && ng > 1 && hipEventRecord(bt->fork, bt->stream) != hipSuccess)
                st = LLGX_E_HIP, bt->err = "event record failed";
            for (size_t g = 0; g < ng && st == LLGX_OK; ++g) {
                Ctx* c = bt->groups[g];
                if (g > 0) {
                    if (hipStreamWaitEvent(bt->gstreams[g - 1], bt->fork, 0) != hipSuccess) {
                        st = LLGX_E_HIP;
                        bt->err = "stream wait failed";
                        break;
                    }
                    c->stream = bt->gstreams[g - 1];
                }
                st = enqueue_attempt<T>(c, plans[g]);
                if (st) bt->err = c->err;
                if (g > 0) {
                    if (st == LLGX_OK && hipEventRecord(bt->joins[g - 1], c->stream) != hipSuccess)
                        st = LLGX_E_HIP, bt->err = "event record failed";
                    c->stream = bt->stream;
                }
            }
            for (size_t g = 1; g < ng && st == LLGX_OK; ++g)
                if (hipStreamWaitEvent(bt->stream, bt->joins[g - 1], 0) != hipSuccess)
                    st = LLGX_E_HIP, bt->err = "stream wait failed";
            hipError_t e2 = hipStreamEndCapture(bt->stream, &gr);
            if (st) return st;
            if (e2 != hipSuccess) {
                bt->err = std::string("graph capture failed: ") + hipGetErrorString(e2);
                return LLGX_E_HIP;
            }
            hipGraphExec_t ge;
            if (hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0) != hipSuccess) {
                (void)hipGraphDestroy(gr);
                bt->err = "graph instantiation failed";
                return LLGX_E_HIP;
            }
            (void)hipGraphDestroy(gr);
            it = bt->graphs.emplace(keys, ge).first;
            bt->last_jobs = 0;
            bt->last_kernels = -1;
        }
        if (hipGraphLaunch(it->second, bt->stream) != hipSuccess) {
            bt->err = "graph launch failed";
            return LLGX_E_HIP;
        }
        for (size_t g = 0; g < bt->groups.size(); ++g) {
            Ctx* c = bt->groups[g];
            const Plan& pl = plans[g];
            c->n_exact += 1 + (pl.extrap ? 0 : pl.tab->S - 1);
            c->n_extrap += pl.extrap ? pl.tab->S - 1 : 0;
            llgx_status st = commit<T>(c, pl, s->h);
            if (st) return st;
            if (s->renormalize && launch_renorm<T>(c->stream, c->ncell, c->nb, (T*)c->M, c->p.Ms) != hipSuccess) {
                bt->err = "renormalisation launch failed";
                return LLGX_E_HIP;
            }
            c->h_next = s->h;
        }
    }
    return LLGX_OK;
}

}  // namespace llgx

extern "C" {

llgx_status llgx_create(const llgx_problem* p, int32_t precision, int32_t spectral, void* hip_stream,
                        llgx_handle* out) {
    g_create_error.clear();
    if (!p || !out) {
        g_create_error = "null argument";
        return LLGX_E_ARG;
    }
    Ctx* c = nullptr;
    llgx_status st = create_ctx(p, 1, nullptr, precision, spectral, hip_stream, &c, g_create_error);
    *out = (llgx_handle)c;
    return st;
}

llgx_status llgx_batch_create(int32_t n, const llgx_problem* problems, int32_t precision, int32_t spectral,
                              void* hip_stream, llgx_batch* out) {
    g_create_error.clear();
    if (!problems || !out || n < 1) {
        g_create_error = "null argument or n < 1";
        return LLGX_E_ARG;
    }
    *out = nullptr;
    Batch* bt = new Batch();
    bt->stream = (hipStream_t)hip_stream;
    std::vector<std::vector<int>> members;
    for (int i = 0; i < n; ++i) {
        int g = -1;
        for (size_t q = 0; q < members.size(); ++q)
            if (same_material(problems[members[q][0]], problems[i])) g = (int)q;
        if (g < 0) {
            g = (int)members.size();
            members.push_back({});
        }
        bt->where.push_back({g, (int)members[g].size()});
        members[g].push_back(i);
    }
    for (auto& mem : members) {
        std::vector<double> ha;
        for (int i : mem)
            for (int c = 0; c < 3; ++c) ha.push_back(problems[i].Ha[c]);
        Ctx* c = nullptr;
        llgx_status st = create_ctx(&problems[mem[0]], (int)mem.size(), ha.data(), precision, spectral,
                                    hip_stream, &c, g_create_error);
        if (st) {
            for (Ctx* q : bt->groups) {
                release(q);
                delete q;
            }
            delete bt;
            return st;
        }
        bt->groups.push_back(c);
    }
    *out = (llgx_batch)bt;
    return LLGX_OK;
}

void llgx_batch_destroy(llgx_batch b) {
    if (!b) return;
    Batch* bt = (Batch*)b;
    (void)hipStreamSynchronize(bt->stream);
    for (auto& kv : bt->graphs) (void)hipGraphExecDestroy(kv.second);
    for (void* p : bt->tables) (void)hipFree(p);
    for (auto e : bt->joins) (void)hipEventDestroy(e);
    for (auto e : bt->cap_events) (void)hipEventDestroy(e);
    if (bt->fork) (void)hipEventDestroy(bt->fork);
    for (auto st : bt->gstreams) (void)hipStreamDestroy(st);
    for (Ctx* c : bt->groups) {
        release(c);
        delete c;
    }
    delete bt;
}

const char* llgx_batch_last_error(llgx_batch b) {
    if (!b) return g_create_error.c_str();
    return ((Batch*)b)->err.c_str();
}

llgx_status llgx_batch_precompute_demag(llgx_batch b) {
    if (!b) return LLGX_E_ARG;
    Batch* bt = (Batch*)b;
    for (Ctx* c : bt->groups) {
        if (c->have_kernel) continue;
        llgx_status st = precompute(c);
        if (st) {
            bt->err = c->err;
            return st;
        }
    }
    return LLGX_OK;
}

static llgx_status batch_copy(llgx_batch b, int32_t i, const void* src, void* dst_or_null, bool set) {
    Batch* bt = (Batch*)b;
    if (i < 0 || i >= (int)bt->where.size()) {
        bt->err = "sample index out of range";
        return LLGX_E_ARG;
    }
    Ctx* c = bt->groups[bt->where[i].first];
    const size_t bytes = 3 * (size_t)c->ncell * c->tsz;
    char* base = (char*)c->M + (size_t)bt->where[i].second * bytes;
    hipError_t e;
    if (set) {
        e = hipMemcpyAsync(base, src, bytes, hipMemcpyDeviceToDevice, c->stream);
        c->hist.clear();  // the group's Eq. (6) history no longer matches its state
        c->fsal_valid = false;
        c->abm_have_f = c->abm_have_prev = false;
        c->have_m = true;
        if (e == hipSuccess && detect_empty(c) != LLGX_OK) {
            bt->err = c->err;
            return LLGX_E_HIP;
        }
    } else {
        e = hipMemcpyAsync(dst_or_null, base, bytes, hipMemcpyDeviceToDevice, c->stream);
    }
    if (e != hipSuccess) {
        bt->err = std::string("copy failed: ") + hipGetErrorString(e);
        return LLGX_E_HIP;
    }
    return LLGX_OK;
}

llgx_status llgx_batch_set_m(llgx_batch b, int32_t i, const void* M_dev) {
    if (!b || !M_dev) return LLGX_E_ARG;
    return batch_copy(b, i, M_dev, nullptr, true);
}

llgx_status llgx_batch_get_m(llgx_batch b, int32_t i, void* M_dev) {
    if (!b || !M_dev) return LLGX_E_ARG;
    return batch_copy(b, i, nullptr, M_dev, false);
}

llgx_status llgx_batch_run_fixed(llgx_batch b, const llgx_stepper* s, int64_t nsteps, int32_t use_graph) {
    if (!b) return LLGX_E_ARG;
    Batch* bt = (Batch*)b;
    if (bt->groups.empty()) return LLGX_E_STATE;
    return bt->groups[0]->prec == LLGX_F32 ? batch_run_fixed<float>(bt, s, nsteps, use_graph)
                                           : batch_run_fixed<double>(bt, s, nsteps, use_graph);
}

llgx_status llgx_batch_step(llgx_batch b, const llgx_stepper* s, llgx_step_info* info) {
    if (!b) return LLGX_E_ARG;
    Batch* bt = (Batch*)b;
    if (bt->groups.empty()) return LLGX_E_STATE;
    return bt->groups[0]->prec == LLGX_F32 ? batch_step<float>(bt, s, info) : batch_step<double>(bt, s, info);
}

llgx_status llgx_batch_autotune(llgx_batch b, int32_t reps) {
    if (!b) return LLGX_E_ARG;
    Batch* bt = (Batch*)b;
    for (Ctx* g : bt->groups) {
        llgx_status st = tune_ctx(g, reps, nullptr);
        if (st) {
            bt->err = g->err;
            return st;
        }
    }
    (void)hipStreamSynchronize(bt->stream);
    for (auto& kv : bt->graphs) (void)hipGraphExecDestroy(kv.second);
    bt->graphs.clear();
    for (void* p : bt->tables) (void)hipFree(p);
    bt->tables.clear();
    for (auto e : bt->cap_events) (void)hipEventDestroy(e);
    bt->cap_events.clear();
    return LLGX_OK;
}

llgx_status llgx_batch_set_launch(llgx_batch b, int32_t mode) {
    if (!b) return LLGX_E_ARG;
    Batch* bt = (Batch*)b;
    if (mode != LLGX_BATCH_JOBS && mode != LLGX_BATCH_STREAMS) {
        bt->err = "unknown batch launch mode";
        return LLGX_E_ARG;
    }
    if (mode != bt->mode) {
        (void)hipStreamSynchronize(bt->stream);
        for (auto& kv : bt->graphs) (void)hipGraphExecDestroy(kv.second);
        bt->graphs.clear();
        for (void* p : bt->tables) (void)hipFree(p);
        bt->tables.clear();
        for (auto e : bt->cap_events) (void)hipEventDestroy(e);
        bt->cap_events.clear();
        bt->mode = mode;
    }
    return LLGX_OK;
}

llgx_status llgx_batch_launch_info(llgx_batch b, int32_t* job_table, int32_t* kernels_per_step) {
    if (!b) return LLGX_E_ARG;
    Batch* bt = (Batch*)b;
    if (job_table) *job_table = bt->last_jobs;
    if (kernels_per_step) *kernels_per_step = bt->last_kernels;
    return LLGX_OK;
}

llgx_status llgx_batch_info(llgx_batch b, int32_t* ngroups, int64_t* total_cells, double* t) {
    if (!b) return LLGX_E_ARG;
    Batch* bt = (Batch*)b;
    if (ngroups) *ngroups = (int32_t)bt->groups.size();
    if (total_cells) {
        int64_t n = 0;
        for (Ctx* c : bt->groups) n += c->ncell * c->nb;
        *total_cells = n;
    }
    if (t) *t = bt->groups.empty() ? 0.0 : bt->groups[0]->t;
    return LLGX_OK;
}

void llgx_destroy(llgx_handle h) {
    if (!h) return;
    Ctx* c = (Ctx*)h;
    (void)hipStreamSynchronize(c->stream);
    release(c);
    delete c;
}

llgx_status llgx_precompute_demag(llgx_handle h) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (c->have_kernel && c->octant) return LLGX_OK;
    return precompute(c);
}

llgx_status llgx_set_demag_tensor(llgx_handle h, const double* N_host) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!N_host) return c->fail(LLGX_E_ARG, "null tensor");
    const long nfull = 6L * (2 * c->nx - 1) * (2 * c->ny - 1) * (2 * c->nz - 1);
    std::vector<double> full(N_host, N_host + nfull);
    const long o = (((long)(c->nz - 1) * (2 * c->ny - 1) + (c->ny - 1)) * (2 * c->nx - 1)) + (c->nx - 1);
    const long cs = (long)(2 * c->nz - 1) * (2 * c->ny - 1) * (2 * c->nx - 1);
    for (int i = 0; i < 3; ++i) c->n00[i] = full[i * cs + o];
    c->hist.clear();
    c->fsal_valid = false;
    c->abm_have_f = c->abm_have_prev = false;
    return c->prec == LLGX_F32 ? kernel_from_octant_or_real<float>(c, &full)
                               : kernel_from_octant_or_real<double>(c, &full);
}

llgx_status llgx_get_demag_tensor(llgx_handle h, double* N_host) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!N_host) return c->fail(LLGX_E_ARG, "null output");
    if (!c->octant) return c->fail(LLGX_E_STATE, "tensor not computed on the device (llgx_precompute_demag)");
    HIPCHK(c, hipMemcpyAsync(N_host, c->octant, 6L * c->ncell * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LLGX_OK;
}

llgx_status llgx_self_tensor(llgx_handle h, double n00[3]) {
    if (!h || !n00) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!c->have_kernel) return c->fail(LLGX_E_STATE, "demag kernel not computed");
    for (int i = 0; i < 3; ++i) n00[i] = c->n00[i];
    return LLGX_OK;
}

llgx_status llgx_set_m(llgx_handle h, const void* M_dev) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!M_dev) return c->fail(LLGX_E_ARG, "null M");
    HIPCHK(c, hipMemcpyAsync(c->M, M_dev, 3 * (size_t)c->ncell * c->nb * c->tsz, hipMemcpyDeviceToDevice, c->stream));
    llgx_status st = detect_empty(c);
    if (st) return st;
    c->have_m = true;
    c->hist.clear();
    c->fsal_valid = false;
    c->abm_have_f = c->abm_have_prev = false;
    return LLGX_OK;
}

llgx_status llgx_get_m(llgx_handle h, void* M_dev) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!M_dev) return c->fail(LLGX_E_ARG, "null M");
    if (!c->have_m) return c->fail(LLGX_E_STATE, "magnetization not set");
    HIPCHK(c, hipMemcpyAsync(M_dev, c->M, 3 * (size_t)c->ncell * c->nb * c->tsz, hipMemcpyDeviceToDevice, c->stream));
    return LLGX_OK;
}

static llgx_status field_call(llgx_handle h, const void* M_dev, void* out_dev, int mode) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!M_dev || !out_dev) return c->fail(LLGX_E_ARG, "null pointer");
    if (!c->have_kernel) return c->fail(LLGX_E_STATE, "demag kernel not computed (llgx_precompute_demag)");
    XinvOut out{nullptr, nullptr, nullptr};
    if (mode == XINV_RHS)
        out.f = out_dev;
    else
        out.h = out_dev;
    llgx_status st = detect_empty(c, M_dev, 1);
    if (st) return st;
    c->field_input = true;
    if (c->prec == LLGX_F32)
        st = eval_exact<float>(c, plain<float>(M_dev), nullptr, mode, (const float*)M_dev, out);
    else
        st = eval_exact<double>(c, plain<double>(M_dev), nullptr, mode, (const double*)M_dev, out);
    c->field_input = false;
    return st;
}

llgx_status llgx_demag(llgx_handle h, const void* M_dev, void* H_dev) { return field_call(h, M_dev, H_dev, XINV_DEMAG); }
llgx_status llgx_heff(llgx_handle h, const void* M_dev, void* H_dev) { return field_call(h, M_dev, H_dev, XINV_HEFF); }
llgx_status llgx_rhs(llgx_handle h, const void* M_dev, void* F_dev) { return field_call(h, M_dev, F_dev, XINV_RHS); }

llgx_status llgx_demag_noalloc(llgx_handle h, const void* M_dev, void* H_dev) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!M_dev || !H_dev) return c->fail(LLGX_E_ARG, "null pointer");
    if (!c->have_kernel) return c->fail(LLGX_E_STATE, "demag kernel not computed (llgx_precompute_demag)");
    if (!c->noalloc) return c->fail(LLGX_E_STATE, "no scratch address on this device");
    // layout: [0, 256) the empty-cell flag, then spectrum A, then spectrum B
    const size_t cbytes = c->spectral == LLGX_SPEC_NATIVE ? 2 * c->tsz : 4;
    const size_t bytesA = 3 * (size_t)c->nz * c->ny * c->SX * cbytes * c->nb;
    const size_t bytesB = c->Py > 1 ? 3 * (size_t)c->nz * c->Py * c->SX * cbytes * c->nb : 0;
    const size_t offA = 256, offB = offA + (bytesA + 255) / 256 * 256;
    const size_t need = offB + bytesB;
    if (need > (size_t)LLGX_NOALLOC_SCRATCH_BYTES)
        return c->fail(LLGX_E_ARG, "mesh needs %zu bytes of scratch; llgx_demag_noalloc has %zu", need,
                       (size_t)LLGX_NOALLOC_SCRATCH_BYTES);
    char* base = (char*)c->noalloc;
    int* flag = (int*)base;
    HIPCHK(c, launch_fill_int(c->stream, flag, 1, 0));
    if (c->prec == LLGX_F32)
        HIPCHK(c, launch_detect_empty<float>(c->stream, c->ncell, c->nb, (const float*)M_dev, flag));
    else
        HIPCHK(c, launch_detect_empty<double>(c->stream, c->ncell, c->nb, (const double*)M_dev, flag));
    c->empty_use = flag;
    c->spec_use[0] = base + offA;
    c->spec_use[1] = bytesB ? base + offB : nullptr;
    XinvOut out{H_dev, nullptr, nullptr};
    llgx_status st = c->prec == LLGX_F32
                         ? eval_exact<float>(c, plain<float>(M_dev), nullptr, XINV_DEMAG, (const float*)M_dev, out)
                         : eval_exact<double>(c, plain<double>(M_dev), nullptr, XINV_DEMAG, (const double*)M_dev, out);
    c->empty_use = nullptr;
    c->spec_use[0] = c->spec_use[1] = nullptr;
    return st;
}

llgx_status llgx_step(llgx_handle h, const llgx_stepper* s, llgx_step_info* info) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    return c->prec == LLGX_F32 ? do_step<float>(c, s, info) : do_step<double>(c, s, info);
}

llgx_status llgx_run_fixed(llgx_handle h, const llgx_stepper* s, int64_t nsteps, int32_t use_graph,
                           llgx_step_info* info) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (nsteps < 0) return c->fail(LLGX_E_ARG, "nsteps < 0");
    return c->prec == LLGX_F32 ? do_run_fixed<float>(c, s, nsteps, use_graph, info)
                               : do_run_fixed<double>(c, s, nsteps, use_graph, info);
}

llgx_status llgx_run(llgx_handle h, const llgx_stepper* s, double t_end, double sample_dt, double* mavg_host,
                     int64_t cap, int64_t* nsamples) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!s) return c->fail(LLGX_E_ARG, "null stepper");
    return c->prec == LLGX_F32 ? do_run<float>(c, s, t_end, sample_dt, mavg_host, cap, nsamples)
                               : do_run<double>(c, s, t_end, sample_dt, mavg_host, cap, nsamples);
}

llgx_status llgx_profile(llgx_handle h, int32_t enable) {
    if (!h) return LLGX_E_ARG;
    ((Ctx*)h)->prof = enable != 0;
    return LLGX_OK;
}

llgx_status llgx_profile_read(llgx_handle h, double ms[LLGX_K_COUNT], int64_t launches[LLGX_K_COUNT]) {
    if (!h || !ms || !launches) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    for (int k = 0; k < LLGX_K_COUNT; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    for (auto& m : c->marks) {
        float t = 0.f;
        HIPCHK(c, hipEventElapsedTime(&t, m.a, m.b));
        ms[m.kind] += t;
        launches[m.kind]++;
        c->spare.push_back(m.a);
        c->spare.push_back(m.b);
    }
    c->marks.clear();
    return LLGX_OK;
}

llgx_status llgx_get_time(llgx_handle h, double* t, double* h_next) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (t) *t = c->t;
    if (h_next) *h_next = c->h_next;
    return LLGX_OK;
}

llgx_status llgx_set_time(llgx_handle h, double t) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    c->t = t;
    c->hist.clear();
    c->fsal_valid = false;
    c->abm_have_f = c->abm_have_prev = false;
    return LLGX_OK;
}

llgx_status llgx_autotune(llgx_handle h, int32_t reps, double us_out[5]) {
    if (!h) return LLGX_E_ARG;
    return tune_ctx((Ctx*)h, reps, us_out);
}

llgx_status llgx_time_passes(llgx_handle h, int32_t reps, double us_out[5]) {
    if (!h || !us_out) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (reps < 1) return c->fail(LLGX_E_ARG, "reps must be >= 1");
    if (!c->have_kernel) return c->fail(LLGX_E_STATE, "demag kernel not computed (llgx_precompute_demag)");
    if (!c->have_m) return c->fail(LLGX_E_STATE, "magnetization not set (llgx_set_m)");
    for (int k = 0; k < 5; ++k) {
        us_out[k] = 0.0;
        if (!pass_exists(c, k)) continue;
        llgx_status st = time_pass_any(c, k, c->var[k], reps, &us_out[k]);
        if (st) return st;
    }
    return LLGX_OK;
}

llgx_status llgx_variant_counts(int32_t n[5]) {
    if (!n) return LLGX_E_ARG;
    for (int k = 0; k < 5; ++k) n[k] = kNumVar[k];
    return LLGX_OK;
}

llgx_status llgx_get_variants(llgx_handle h, int32_t v[5]) {
    if (!h || !v) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    for (int k = 0; k < 5; ++k) v[k] = c->var[k];
    return LLGX_OK;
}

llgx_status llgx_set_variants(llgx_handle h, const int32_t v[5]) {
    if (!h || !v) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    for (int k = 0; k < 5; ++k)
        if (v[k] < 0 || v[k] >= kNumVar[k]) return c->fail(LLGX_E_ARG, "variant %d of pass %d out of range", v[k], k);
    for (int k = 0; k < 5; ++k) c->var[k] = v[k];
    drop_graphs(c);
    return LLGX_OK;
}

llgx_status llgx_tune_export(char* buf, size_t cap, size_t* used) {
    std::string out;
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (const auto& kv : g_tune) {
            char line[512];
            const TuneEntry& e = kv.second;
            snprintf(line, sizeof line,
                     "{\"key\": \"%s\", \"variant\": [%d, %d, %d, %d, %d], \"us\": [%.3f, %.3f, %.3f, %.3f, %.3f]}\n",
                     kv.first.c_str(), e.var[0], e.var[1], e.var[2], e.var[3], e.var[4], e.us[0], e.us[1], e.us[2],
                     e.us[3], e.us[4]);
            out += line;
        }
    }
    if (used) *used = out.size() + 1;
    if (!buf) return LLGX_OK;
    if (cap < out.size() + 1) return LLGX_E_ARG;
    memcpy(buf, out.c_str(), out.size() + 1);
    return LLGX_OK;
}

llgx_status llgx_tune_import(const char* text) {
    if (!text) return LLGX_E_ARG;
    std::map<std::string, TuneEntry> add;
    const char* p = text;
    while (*p) {
        const char* eol = strchr(p, '\n');
        std::string line(p, eol ? (size_t)(eol - p) : strlen(p));
        p = eol ? eol + 1 : p + line.size();
        if (line.find_first_not_of(" \t\r") == std::string::npos) continue;
        char key[160] = {0};
        TuneEntry e{};
        const size_t kp = line.find("\"key\"");
        const size_t vp = line.find("\"variant\"");
        if (kp == std::string::npos || vp == std::string::npos) return LLGX_E_ARG;
        if (sscanf(line.c_str() + kp, "\"key\" : \"%159[^\"]\"", key) != 1 &&
            sscanf(line.c_str() + kp, "\"key\": \"%159[^\"]\"", key) != 1)
            return LLGX_E_ARG;
        if (sscanf(line.c_str() + vp, "\"variant\": [%d, %d, %d, %d, %d]", &e.var[0], &e.var[1], &e.var[2],
                   &e.var[3], &e.var[4]) != 5)
            return LLGX_E_ARG;
        for (int k = 0; k < 5; ++k)
            if (e.var[k] < 0 || e.var[k] >= kNumVar[k]) return LLGX_E_ARG;
        const size_t up = line.find("\"us\"");
        if (up != std::string::npos)
            (void)sscanf(line.c_str() + up, "\"us\": [%lf, %lf, %lf, %lf, %lf]", &e.us[0], &e.us[1], &e.us[2],
                         &e.us[3], &e.us[4]);
        add[key] = e;
    }
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : add) g_tune[kv.first] = kv.second;
    return LLGX_OK;
}

// ---- checkpoint ---------------------------------------------------------
// Host image: header, then M, then the history fields oldest first, then
// (when held) the start derivative F_n (FSAL stage or ABM2), the stored field
// of the current ABM2 start and the ABM2 derivative F_{n-1}.  All arrays in
// the working precision.
struct CkptHeader {
    char magic[8];
    int32_t version, prec, nx, ny, nz, nb;
    int32_t method, p, nhist, fsal_valid;
    int32_t abm_have_f, abm_have_g, abm_have_prev, pad;
    double t, h_next, abm_hprev;
    double hist_t[MAX_HIST];
    int64_t counters[5];
};
static const char kCkptMagic[8] = {'L', 'L', 'G', 'X', 'C', 'K', 'P', '2'};

static size_t ckpt_arrays(const CkptHeader& hd) {
    return 1 + (size_t)hd.nhist + (size_t)(hd.fsal_valid || hd.abm_have_f) + (size_t)hd.abm_have_g +
           (size_t)hd.abm_have_prev;
}

static CkptHeader ckpt_header(const Ctx* c) {
    CkptHeader hd{};
    memcpy(hd.magic, kCkptMagic, 8);
    hd.version = 2;
    hd.prec = c->prec;
    hd.nx = c->nx;
    hd.ny = c->ny;
    hd.nz = c->nz;
    hd.nb = c->nb;
    hd.method = c->cur_method;
    hd.p = c->cur_p;
    hd.nhist = (int32_t)c->hist.size();
    hd.fsal_valid = c->fsal_valid ? 1 : 0;
    hd.abm_have_f = c->abm_have_f ? 1 : 0;
    hd.abm_have_g = (c->abm_have_f && c->cur_p >= 0) ? 1 : 0;
    hd.abm_have_prev = c->abm_have_prev ? 1 : 0;
    hd.t = c->t;
    hd.h_next = c->h_next;
    hd.abm_hprev = c->abm_hprev;
    for (size_t i = 0; i < c->hist.size(); ++i) hd.hist_t[i] = c->hist[i].t;
    hd.counters[0] = c->n_exact;
    hd.counters[1] = c->n_extrap;
    hd.counters[2] = c->n_acc;
    hd.counters[3] = c->n_rej;
    hd.counters[4] = c->n_forced;
    return hd;
}

llgx_status llgx_save_state(llgx_handle h, void* host_buf, size_t cap, size_t* used) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!c->have_m) return c->fail(LLGX_E_STATE, "magnetization not set");
    const CkptHeader hd = ckpt_header(c);
    const size_t vec = 3 * (size_t)c->ncell * c->nb * c->tsz;
    const size_t need = sizeof hd + vec * ckpt_arrays(hd);
    if (used) *used = need;
    if (!host_buf) return LLGX_OK;
    if (cap < need) return c->fail(LLGX_E_ARG, "checkpoint needs %zu bytes, buffer holds %zu", need, cap);
    char* out = (char*)host_buf;
    memcpy(out, &hd, sizeof hd);
    size_t off = sizeof hd;
    auto put = [&](const void* src) -> llgx_status {
        HIPCHK(c, hipMemcpyAsync(out + off, src, vec, hipMemcpyDeviceToHost, c->stream));
        off += vec;
        return LLGX_OK;
    };
    llgx_status st = put(c->M);
    for (size_t i = 0; i < c->hist.size() && !st; ++i) st = put(c->G[c->hist[i].slot]);
    if (!st && (hd.fsal_valid || hd.abm_have_f)) st = put(c->F[0]);
    if (!st && hd.abm_have_g) st = put(c->G[c->abm_slot]);
    if (!st && hd.abm_have_prev) st = put(c->F[2]);
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return LLGX_OK;
}

llgx_status llgx_load_state(llgx_handle h, const void* host_buf, size_t len) {
    if (!h) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    if (!host_buf || len < sizeof(CkptHeader)) return c->fail(LLGX_E_ARG, "checkpoint too short");
    CkptHeader hd;
    memcpy(&hd, host_buf, sizeof hd);
    if (memcmp(hd.magic, kCkptMagic, 8) != 0 || hd.version != 2)
        return c->fail(LLGX_E_ARG, "not a checkpoint of this library");
    if (hd.prec != c->prec || hd.nx != c->nx || hd.ny != c->ny || hd.nz != c->nz || hd.nb != c->nb)
        return c->fail(LLGX_E_ARG, "checkpoint of a %dx%dx%d x%d mesh in precision %d does not fit this handle",
                       hd.nx, hd.ny, hd.nz, hd.nb, hd.prec);
    auto flag = [](int32_t v) { return v == 0 || v == 1; };
    if (hd.nhist < 0 || hd.nhist > MAX_HIST - 1 || !flag(hd.fsal_valid) || !flag(hd.abm_have_f) ||
        !flag(hd.abm_have_g) || !flag(hd.abm_have_prev) || (hd.abm_have_g && !hd.abm_have_f) ||
        (hd.fsal_valid && hd.abm_have_f) || (hd.abm_have_prev && !(hd.abm_hprev > 0)))
        return c->fail(LLGX_E_ARG, "corrupt checkpoint header");
    const size_t vec = 3 * (size_t)c->ncell * c->nb * c->tsz;
    const size_t need = sizeof hd + vec * ckpt_arrays(hd);
    if (len != need) return c->fail(LLGX_E_ARG, "checkpoint length %zu, expected %zu", len, need);
    const char* in = (const char*)host_buf;
    size_t off = sizeof hd;
    auto get = [&](void* dst) -> llgx_status {
        HIPCHK(c, hipMemcpyAsync(dst, in + off, vec, hipMemcpyHostToDevice, c->stream));
        off += vec;
        return LLGX_OK;
    };
    llgx_status st = get(c->M);
    c->hist.clear();
    for (int i = 0; i < hd.nhist && !st; ++i) {
        st = get(c->G[i]);
        c->hist.push_back({hd.hist_t[i], i});
    }
    if (!st && (hd.fsal_valid || hd.abm_have_f)) st = get(c->F[0]);
    if (!st && hd.abm_have_g) st = get(c->G[hd.nhist]);
    if (!st && hd.abm_have_prev) st = get(c->F[2]);
    if (!st) st = detect_empty(c);
    if (st) return st;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->fsal_valid = hd.fsal_valid != 0;
    c->abm_have_f = hd.abm_have_f != 0;
    c->abm_have_prev = hd.abm_have_prev != 0;
    c->abm_hprev = hd.abm_hprev;
    c->abm_slot = hd.nhist;
    c->cur_method = hd.method;
    c->cur_p = hd.p;
    c->t = hd.t;
    c->h_next = hd.h_next;
    c->n_exact = hd.counters[0];
    c->n_extrap = hd.counters[1];
    c->n_acc = hd.counters[2];
    c->n_rej = hd.counters[3];
    c->n_forced = hd.counters[4];
    c->have_m = true;
    return LLGX_OK;
}

llgx_status llgx_counters(llgx_handle h, int64_t out[5]) {
    if (!h || !out) return LLGX_E_ARG;
    Ctx* c = (Ctx*)h;
    out[0] = c->n_exact;
    out[1] = c->n_extrap;
    out[2] = c->n_acc;
    out[3] = c->n_rej;
    out[4] = c->n_forced;
    return LLGX_OK;
}

}  // extern "C"
