// C-ABI layer of the vkmg library: context, multigrid V-cycle orchestration
// (paper, Algorithm 1) and restarted flexible GMRES (paper, section "Overall
// solver performance"; Saad's flexible variant with right preconditioning).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>
#include <memory>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "../../include/vkmg.h"
#include "kernels.h"
#include "vkmg_internal.h"

using namespace vkmg;

namespace {

thread_local std::string g_last_error;

vkmg_status fail(vkmg_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

#define VKMG_HIP(call)                                                                  \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? VKMG_ERR_OUT_OF_MEMORY : VKMG_ERR_HIP, \
                        std::string(#call) + ": " + hipGetErrorString(e_));             \
    } while (0)

struct LevelBuf {
    Geom g;
    void* x = nullptr;  // MG precision
    void* b = nullptr;
    void* r = nullptr;
    void* x2 = nullptr;    // x + prolonged coarse correction (levels above the coarsest)
    void* W = nullptr;     // patch-operator table, MG precision (relaxed levels)
    void* dbuf = nullptr;  // boundary-patch corrections (relaxed levels)
    void* bs = nullptr;    // Braess-Sarazin scratch: Schur rhs, dp, B^T dp (relaxed levels)
    void* nu = nullptr;    // per-element viscosity, MG precision (variable-viscosity contexts)
};

}  // namespace

// Device scratch of vkmg_vanka_update_noalloc: the patch corrections of one
// Vanka update (the boundary patches', or every patch's for a per-element
// viscosity), which vkmg_vanka_update keeps in a buffer allocated at setup.
// Each GPU holds its own copy until the process ends.  Host code never
// passes `scratch` itself to a kernel: its device address comes from
// hipGetSymbolAddress, per device (noalloc_scratch below).
constexpr size_t kNoAllocScratchBytes = size_t(4) << 20;
static __device__ __align__(256) double scratch[kNoAllocScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on `device`, which must be the current
// device; looked up once per device (at the first setup on it).
vkmg_status noalloc_scratch(int device, void** out) {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0 || device >= kMaxDevices)
        return fail(VKMG_ERR_UNSUPPORTED, "setup: device index beyond the scratch table");
    if (!g_scratch_addr[device]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(VKMG_ERR_HIP, std::string("setup: hipGetSymbolAddress(scratch): ") +
                                          hipGetErrorString(e));
        g_scratch_addr[device] = p;
    }
    *out = g_scratch_addr[device];
    return VKMG_OK;
}

}  // namespace

struct vkmg_ctx {
    int device = 0;
    int L = 0;
    vkmg_options opt{};
    std::vector<LevelBuf> lev;
    double* C = nullptr;  // coarse bordered inverse (n0 x n0), FP64
    void* mtab = nullptr; // matrix-instruction operands of the interior operator (MG precision)
    // FP64 work vectors of the finest level
    double* r64 = nullptr;
    double* w64 = nullptr;
    double* part = nullptr;   // dot partials
    double* hdev = nullptr;   // coefficients (device)
    double* hhost = nullptr;  // pinned host mirror
    double* gstat = nullptr;  // FGMRES: per-system summaries (8 each), then cycle init values
    double* hstat = nullptr;  // pinned: two step summaries and the init values (8 per system each)
    hipEvent_t step_done[2] = {nullptr, nullptr};  // coefficient copies of Arnoldi steps
    // FGMRES basis
    double* V = nullptr;
    double* Z = nullptr;
    int basis_cap = 0;
    // timing
    int32_t timing_mask = 0;
    struct EventPair {
        hipEvent_t start, stop;
        int level;  // -1 for launches not tied to a level (Krylov vectors)
    };
    std::vector<EventPair> events[VKMG_KERNEL_COUNT];
    std::vector<void*> allocations;
    void* noalloc = nullptr;  // device address of `scratch` on this context's device
    vkmg_tuning tune{};       // launch shapes per level size (vkmg_set_tuning)
    // executable graphs of the Arnoldi steps (index j), valid for the
    // current basis allocation; captured on a private stream
    std::vector<hipGraphExec_t> step_graphs;
    int graphs_scheme = -1;  // orthogonalisation scheme the graphs were captured for
    hipStream_t capture_stream = nullptr;

    size_t esize() const { return opt.mg_precision == VKMG_FP32 ? 4 : 8; }
    int nb() const { return opt.batch; }
    bool variable = false;     // per-element viscosity ("simple" Vanka, per-patch inverses)
    double* nu64 = nullptr;    // finest-level per-element viscosity, FP64 (FGMRES residuals)
    template <typename T>
    const T* nu_of(int l) const { return static_cast<const T*>(lev[l].nu); }
    const Geom& top() const { return lev.back().g; }
};

namespace {

constexpr int kHostScratch = 2048;  // doubles per system in hdev and the pinned hhost
static_assert(kHostScratch >= GivensLayout::kSize + 32, "coefficient area holds the Givens state");
// largest restart length orthogonalised by the delayed scheme (its
// kernels hold up to 32 basis coefficients in registers)
constexpr int kDelayedMaxRestart = 32;

// Brackets one kernel launch with events when the class is being timed.
struct Timed {
    vkmg_ctx* c;
    int cls;
    hipStream_t s;
    int level;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    Timed(vkmg_ctx* ctx, int k, hipStream_t st, int lev = -1) : c(ctx), cls(k), s(st), level(lev) {
        if (c->timing_mask & (1 << cls)) {
            (void)hipEventCreate(&e0);
            (void)hipEventCreate(&e1);
            (void)hipEventRecord(e0, s);
        }
    }
    ~Timed() {
        if (e0) {
            (void)hipEventRecord(e1, s);
            c->events[cls].push_back({e0, e1, level});
        }
    }
};

void drop_graphs(vkmg_ctx* c) {
    for (hipGraphExec_t g : c->step_graphs)
        if (g) (void)hipGraphExecDestroy(g);
    c->step_graphs.clear();
}

vkmg_status alloc(vkmg_ctx* c, void** p, size_t bytes) {
    VKMG_HIP(hipMalloc(p, bytes < 256 ? 256 : bytes));
    c->allocations.push_back(*p);
    return VKMG_OK;
}

void free_all(vkmg_ctx* c) {
    for (void* p : c->allocations) (void)hipFree(p);
    c->allocations.clear();
    if (c->hhost) (void)hipHostFree(c->hhost);
    c->hhost = nullptr;
    if (c->hstat) (void)hipHostFree(c->hstat);
    c->hstat = nullptr;
    for (auto& e : c->step_done) {
        if (e) (void)hipEventDestroy(e);
        e = nullptr;
    }

    for (auto& v : c->events)
        for (auto& e : v) {
            (void)hipEventDestroy(e.start);
            (void)hipEventDestroy(e.stop);
        }
    drop_graphs(c);
    if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    c->capture_stream = nullptr;
}

hipStream_t as_stream(void* s) { return reinterpret_cast<hipStream_t>(s); }

vkmg_layout layout_of_geom(const Geom& g) {
    vkmg_layout l;
    l.n = g.n;
    l.n_vel = 2 * g.nq2;
    l.n_pres = g.nq1;
    l.off_ux = 0;
    l.off_uy = g.nq2;
    l.off_p = 2 * g.nq2;
    l.q2_side = g.s2;
    l.q1_side = g.s1;
    l.n_elem = g.N;
    return l;
}

// ------------------------------------------------------------------ MG steps

// FP64 tile kernel with half of a patch parked in LDS on this level.
template <typename T>
bool parked(const vkmg_ctx* c, int N) {
    return sizeof(T) == 8 && N >= c->tune.park_min_n;
}

// One sweep on level l: r = b - A x, then x += corrections (in place).
// With x_zero the iterate is known to be zero, so r = b and the update
// writes every DoF of x without reading it.  With xin given, L.r already
// holds b - A xin and the update writes xin + corrections to x.
template <typename T>
void sweep_t(vkmg_ctx* c, int l, const T* b, T* x, bool x_zero, hipStream_t s,
             bool vanka = false, const T* xin = nullptr) {
    LevelBuf& L = c->lev[l];
    const T* r = b;
    if (xin) {
        r = static_cast<const T*>(L.r);
    } else if (!x_zero) {
        Timed t(c, VKMG_KERNEL_RESIDUAL, s, l);
        launch_residual<T, T>(L.g, b, x, static_cast<T*>(L.r), 0, s, c->nb(), c->nu_of<T>(l));
        r = static_cast<const T*>(L.r);
        xin = x;
    }
    Timed t(c, VKMG_KERNEL_VANKA, s, l);
    if (c->variable) {
        launch_vanka_simple<T>(L.g, r, xin, x, static_cast<const T*>(L.W),
                               static_cast<T*>(L.dbuf), s, c->nb());
        return;
    }
    if (!vanka && c->opt.relaxation == VKMG_RELAX_BRAESS_SARAZIN) {
        const int64_t np = L.g.nq1 * c->nb();
        T* prhs = static_cast<T*>(L.bs);
        launch_bs_relax<T>(L.g, r, xin, x, prhs, prhs + np, prhs + 2 * np, c->opt.bs_t,
                           c->opt.bs_omega, c->opt.bs_jacobi_weight, c->opt.bs_jacobi_sweeps, s,
                           c->nb());
        return;
    }
    launch_vanka_boundary<T>(L.g, r, static_cast<const T*>(L.W), static_cast<T*>(L.dbuf), s,
                             c->nb(), c->tune.boundary_per_wave);
    Timed tt(c, VKMG_KERNEL_VANKA_TILE, s, l);
    launch_vanka_tiles<T>(L.g, r, xin, x, static_cast<const T*>(c->mtab),
                          static_cast<const T*>(L.dbuf), c->opt.omega,
                          c->opt.interior_apply == VKMG_APPLY_MATRIX, s, c->nb(),
                          parked<T>(c, L.g.N));
}

// b_{l-1} = P^T (b - A_l x): the residual, then the restriction.
template <typename T>
void restrict_residual_t(vkmg_ctx* c, int l, const T* b, const T* x, T* bc, hipStream_t s) {
    LevelBuf& L = c->lev[l];
    LevelBuf& Lc = c->lev[l - 1];
    T* r = static_cast<T*>(L.r);
    {
        Timed t(c, VKMG_KERNEL_RESIDUAL, s, l);
        launch_residual<T, T>(L.g, b, x, r, 0, s, c->nb(), c->nu_of<T>(l));
    }
    Timed t(c, VKMG_KERNEL_TRANSFER, s, l);
    launch_restrict<T>(L.g, Lc.g, r, bc, s, c->nb());
}

// Whether the V-cycle sweeps of level l run as single fused launches.
bool fused_sweeps(const vkmg_ctx* c, int l) {
    const int N = c->lev[l].g.N;
    return c->opt.relaxation == VKMG_RELAX_VANKA && !c->variable &&
           c->opt.interior_apply == VKMG_APPLY_VECTOR && c->opt.nu_pre >= 1 &&
           c->opt.nu_post >= 1 && N >= vanka_fused_min_n() && N <= c->tune.fused_sweep_max_n;
}

template <typename T>
void mg_t(vkmg_ctx* c, int l, const T* b, T* x, hipStream_t s);

// MG(l, b) with every sweep of level l fused into one launch.  The fused
// sweep writes a buffer other than the one it reads, so the iterates
// alternate between x and the level's x2, arranged so that the last sweep
// writes x; the coarse-grid correction is added in place to the last
// pre-smoothed iterate.  Same results as the unfused form.
template <typename T>
void mg_fused_t(vkmg_ctx* c, int l, const T* b, T* x, hipStream_t s) {
    LevelBuf& L = c->lev[l];
    LevelBuf& Lc = c->lev[l - 1];
    T* const x2 = static_cast<T*>(L.x2);
    const T* const W = static_cast<const T*>(L.W);
    const int S = c->opt.nu_pre + c->opt.nu_post;
    auto out = [&](int k) { return ((S - k) % 2 == 0) ? x : x2; };
    T* cur = nullptr;  // x = 0
    for (int k = 1; k <= c->opt.nu_pre; ++k) {
        Timed t(c, VKMG_KERNEL_VANKA, s, l);
        launch_vanka_fused<T>(L.g, b, cur, out(k), W, c->opt.omega, s, c->nb());
        cur = out(k);
    }
    T* bc = static_cast<T*>(Lc.b);
    T* xc = static_cast<T*>(Lc.x);
    restrict_residual_t<T>(c, l, b, cur, bc, s);
    if (l - 1 == 0) {
        Timed t(c, VKMG_KERNEL_COARSE, s, 0);
        launch_coarse_gemv<T>(Lc.g.n, c->C, bc, xc, s, c->nb());
    } else {
        mg_t<T>(c, l - 1, bc, xc, s);
    }
    {
        Timed t(c, VKMG_KERNEL_TRANSFER, s, l);
        launch_prolong_add<T>(L.g, Lc.g, xc, cur, s, c->nb());
    }
    for (int k = c->opt.nu_pre + 1; k <= S; ++k) {
        Timed t(c, VKMG_KERNEL_VANKA, s, l);
        launch_vanka_fused<T>(L.g, b, cur, out(k), W, c->opt.omega, s, c->nb());
        cur = out(k);
    }
}

// MG(l, b) of Algorithm 1 with zero initial guess, result in x.
template <typename T>
void mg_t(vkmg_ctx* c, int l, const T* b, T* x, hipStream_t s) {
    if (fused_sweeps(c, l)) {
        mg_fused_t<T>(c, l, b, x, s);
        return;
    }
    LevelBuf& L = c->lev[l];
    LevelBuf& Lc = c->lev[l - 1];
    bool x_zero = true;
    for (int i = 0; i < c->opt.nu_pre; ++i) {
        sweep_t<T>(c, l, b, x, x_zero, s);
        x_zero = false;
    }
    T* bc = static_cast<T*>(Lc.b);
    T* xc = static_cast<T*>(Lc.x);
    if (x_zero) {
        launch_fill_zero<T>(x, L.g.n * c->nb(), s);
        Timed t(c, VKMG_KERNEL_TRANSFER, s, l);
        launch_restrict<T>(L.g, Lc.g, b, bc, s, c->nb());
    } else {
        restrict_residual_t<T>(c, l, b, x, bc, s);
    }
    if (l - 1 == 0) {
        Timed t(c, VKMG_KERNEL_COARSE, s, 0);
        launch_coarse_gemv<T>(Lc.g.n, c->C, bc, xc, s, c->nb());
    } else {
        mg_t<T>(c, l - 1, bc, xc, s);
    }
    // the coarse-grid correction inside the next residual (FP32: always;
    // FP64: up to the tuned size, above which the separate prolongation and
    // residual kernels are faster)
    const bool fused = sizeof(T) == 4 || L.g.N <= c->tune.fused_prolong_max_n;
    if (c->opt.nu_post == 0 || !fused) {
        Timed t(c, VKMG_KERNEL_TRANSFER, s, l);
        launch_prolong_add<T>(L.g, Lc.g, xc, x, s, c->nb());
    }
    if (c->opt.nu_post == 0) return;
    if (!fused) {
        for (int i = 0; i < c->opt.nu_post; ++i) sweep_t<T>(c, l, b, x, false, s);
        return;
    }
    {  // x + P xc into x2 and its residual in one pass; the first sweep
       // then updates x2 into x
        Timed t(c, VKMG_KERNEL_RESIDUAL, s, l);
        launch_residual_prolong<T>(L.g, Lc.g, b, x, xc, static_cast<T*>(L.x2),
                                   static_cast<T*>(L.r), s, c->nb(), c->nu_of<T>(l));
    }
    sweep_t<T>(c, l, b, x, false, s, false, static_cast<const T*>(L.x2));
    for (int i = 1; i < c->opt.nu_post; ++i) sweep_t<T>(c, l, b, x, false, s);
}

// r32_ready (FP32 multigrid): the top level's b already holds r rounded to
// FP32 (written by the Gram-Schmidt kernel that produced r).
// z32_only (FP32 multigrid): z is left in FP32 in the top level's x and not
// written (launch_apply_widen writes it next to A z).
void vcycle_impl(vkmg_ctx* c, const double* r, double* z, hipStream_t s, bool r32_ready = false,
                 bool z32_only = false) {
    const int top = c->L - 1;
    if (c->opt.mg_precision == VKMG_FP64) {
        mg_t<double>(c, top, r, z, s);
    } else {
        LevelBuf& L = c->lev[top];
        if (!r32_ready)
            launch_cast<double, float>(r, static_cast<float*>(L.b), L.g.n * c->nb(), s);
        mg_t<float>(c, top, static_cast<const float*>(L.b), static_cast<float*>(L.x), s);
        if (!z32_only)
            launch_cast<float, double>(static_cast<const float*>(L.x), z, L.g.n * c->nb(), s);
    }
}

// ---------------------------------------------------------------- Krylov helpers

// Squared norm / dots into hdev[0..k) (device), asynchronous.
void dots_async(vkmg_ctx* c, const double* V, int64_t ldv, int k, const double* w, double* out,
                hipStream_t s) {
    const int64_t n = c->top().n;
    Timed t(c, VKMG_KERNEL_KRYLOV, s);
    launch_mdot_partial(V, ldv, k, w, n, c->part, s);
    launch_reduce_partials(c->part, k, out, s);
}

vkmg_status norm_sync(vkmg_ctx* c, const double* w, double* out, hipStream_t s) {
    dots_async(c, w, 0, 1, w, c->hdev, s);
    VKMG_HIP(hipMemcpyAsync(c->hhost, c->hdev, sizeof(double), hipMemcpyDeviceToHost, s));
    VKMG_HIP(hipStreamSynchronize(s));
    *out = std::sqrt(c->hhost[0]);
    return VKMG_OK;
}

// Basis vectors are stored with a stride rounded up to 64 doubles (512 B),
// so that every vector starts on a cache-line boundary.
int64_t basis_stride(int64_t n) { return (n + 63) / 64 * 64; }

vkmg_status ensure_basis(vkmg_ctx* c, int m) {
    if (m <= c->basis_cap) return VKMG_OK;
    // a basis slot holds the batch's vectors back to back
    const int64_t n = basis_stride(c->top().n * c->nb());
    // captured Arnoldi steps refer to the old basis
    drop_graphs(c);
    // release the old basis (kept in the allocation list until destroy otherwise)
    for (void* p : {static_cast<void*>(c->V), static_cast<void*>(c->Z)}) {
        if (!p) continue;
        auto it = std::find(c->allocations.begin(), c->allocations.end(), p);
        if (it != c->allocations.end()) c->allocations.erase(it);
        (void)hipFree(p);
    }
    c->V = c->Z = nullptr;
    c->basis_cap = 0;
    vkmg_status st = alloc(c, reinterpret_cast<void**>(&c->V), size_t(m + 1) * n * sizeof(double));
    if (st != VKMG_OK) return st;
    st = alloc(c, reinterpret_cast<void**>(&c->Z), size_t(m) * n * sizeof(double));
    if (st != VKMG_OK) return st;
    c->basis_cap = m;
    return VKMG_OK;
}

// Executable graph of Arnoldi step j, captured on the context's private
// stream the first time it is needed (a graph may then be launched on any
// stream, including the legacy default one, which cannot be captured).
template <typename F>
vkmg_status step_graph(vkmg_ctx* c, int j, F&& step) {
    if (int(c->step_graphs.size()) <= j) c->step_graphs.resize(j + 1, nullptr);
    if (c->step_graphs[j]) return VKMG_OK;
    if (!c->capture_stream) {
        hipError_t e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(VKMG_ERR_HIP, std::string("graph stream: ") + hipGetErrorString(e));
    }
    hipError_t e = hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal);
    if (e != hipSuccess) return fail(VKMG_ERR_HIP, std::string("begin capture: ") + hipGetErrorString(e));
    step(j, c->capture_stream);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(c->capture_stream, &graph);
    if (e != hipSuccess || !graph)
        return fail(VKMG_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e));
    hipGraphExec_t exec = nullptr;
    e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(VKMG_ERR_HIP, std::string("instantiate: ") + hipGetErrorString(e));
    c->step_graphs[j] = exec;
    return VKMG_OK;
}

bool check_level(const vkmg_ctx* c, int32_t level, bool relaxed) {
    return c && level >= (relaxed ? 1 : 0) && level < c->L;
}

}  // namespace

namespace {

// Restarted FGMRES with the delayed CGS2 Arnoldi process (restart <= 32)
// for the B >= 1 independent systems of a context.  Each Arnoldi step is
// one batched launch per kernel (V-cycle, operator, the two Gram-Schmidt
// passes) followed by the Givens kernel, which updates every system's
// Hessenberg column, rotations and residual estimate on the device and
// takes the stopping decision there (GivensLayout areas, kHostScratch
// doubles per system in hdev).  The host reads back only two values per
// system and step (estimate, active flag), one step behind the GPU: step
// j+1 is enqueued before the host waits for step j's flags unless every
// active system's estimate, extrapolated at its last rate, may reach the
// tolerance at step j (factor 8 of margin).  A system that has stopped
// rides along with its state frozen until the cycle ends.  At the end of a
// cycle the device solves R y = g and updates x += Z y; the restart
// decision needs the true residual norms (one synchronisation per cycle).
vkmg_status fgmres_delayed(vkmg_ctx* ctx, const double* b, double* x, double rtol, int m,
                           int max_iters, vkmg_info* info, hipStream_t s) {
    using GL = GivensLayout;
    const int B = ctx->nb();
    const Geom& g = ctx->top();
    const int64_t n = g.n;
    const int64_t S = basis_stride(n * B);  // stride of the basis slots
    const int64_t HS = kHostScratch;
    double* r = ctx->r64;
    double* w = ctx->w64;
    double* V = ctx->V;
    double* Z = ctx->Z;
    double* hd = ctx->hdev;
    double* hh = ctx->hhost;
    // compact per-system summaries (8 doubles each): the device's in gstat,
    // the host copies of two consecutive steps in hstat[0..16B), the cycle
    // init values staged in hstat[16B..24B) and copied to gstat[8B..16B)
    double* const gsum = ctx->gstat;
    double* const ginit = ctx->gstat + 8 * B;
    double* const hsum[2] = {ctx->hstat, ctx->hstat + 8 * B};
    double* const hinit = ctx->hstat + 16 * B;

    auto norms = [&](const double* v, std::vector<double>& out) -> vkmg_status {
        {
            Timed t(ctx, VKMG_KERNEL_KRYLOV, s);
            launch_mdot_partial(v, 0, 1, v, n, ctx->part, s, B, n);
            launch_reduce_partials(ctx->part, 1, hd, s, B, HS);
        }
        VKMG_HIP(hipMemcpy2DAsync(hh, HS * 8, hd, HS * 8, 8, B, hipMemcpyDeviceToHost, s));
        VKMG_HIP(hipStreamSynchronize(s));
        for (int k = 0; k < B; ++k) out[k] = std::sqrt(hh[k * HS]);
        return VKMG_OK;
    };
    auto residual = [&]() {
        Timed t(ctx, VKMG_KERNEL_RESIDUAL, s);
        launch_residual<double, double>(g, b, x, r, 0, s, B, ctx->nu64);
    };
    struct Sys {
        double beta0 = 0, beta = 0, target = 0, est = 1, true_rel = 0;
        double est_last = 1, est_prev = 0;  // estimates after the last two steps (this cycle)
        int iters = 0, restarts = 0;
        bool done = false, active = false;
        vkmg_status status = VKMG_OK;
    };
    std::vector<Sys> sys(B);

    residual();
    std::vector<double> nrm(B);
    vkmg_status st = norms(r, nrm);
    if (st != VKMG_OK) return st;
    for (int k = 0; k < B; ++k) {
        Sys& q = sys[k];
        q.beta0 = q.beta = nrm[k];
        q.target = rtol * q.beta0;
        if (!std::isfinite(q.beta0)) {
            q.done = true;
            q.status = VKMG_ERR_NONFINITE;
            q.est = q.true_rel = NAN;
        } else if (q.beta0 == 0.0) {
            q.done = true;
            q.est = q.true_rel = 0.0;
        }
    }
    // FP32 multigrid: the update kernel rounds the next V-cycle input and the
    // apply widens the V-cycle output (as the precision casts, fused)
    const bool fp32_mg = ctx->opt.mg_precision == VKMG_FP32;
    auto step = [&](int j, hipStream_t ss) {
        double* vj = V + int64_t(j) * S;
        double* zj = Z + int64_t(j) * S;
        vcycle_impl(ctx, vj, zj, ss, fp32_mg && j >= 1, fp32_mg);
        {
            Timed t(ctx, VKMG_KERNEL_RESIDUAL, ss);
            if (fp32_mg)
                launch_apply_widen(g, static_cast<const float*>(ctx->lev.back().x), w, zj, ss,
                                   ctx->nu64, B);
            else
                launch_residual<double, double>(g, nullptr, zj, w, 1, ss, B, ctx->nu64);
        }
        Timed t(ctx, VKMG_KERNEL_KRYLOV, ss);
        launch_dcgs_dots(V, S, j, vj, w, n, ctx->part, ss, B, n);
        launch_reduce_partials(ctx->part, 2 * j + 3, hd + GL::kDots, ss, B, HS);
        launch_dcgs_update(V, S, j, hd + GL::kDots, vj, w, V + int64_t(j + 1) * S, n,
                           hd + GL::kCoef, ss, B, n, HS,
                           fp32_mg ? static_cast<float*>(ctx->lev.back().b) : nullptr, hd, gsum);
    };
    const bool use_graphs = ctx->opt.use_graphs != 0 && ctx->timing_mask == 0;
    if (use_graphs && ctx->graphs_scheme != 3) {
        drop_graphs(ctx);
        ctx->graphs_scheme = 3;
    }
    for (auto& e : ctx->step_done)
        if (!e) VKMG_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    auto enqueue_step = [&](int j) -> vkmg_status {
        if (use_graphs) {
            vkmg_status sg = step_graph(ctx, j, step);
            if (sg != VKMG_OK) return sg;
            VKMG_HIP(hipGraphLaunch(ctx->step_graphs[j], s));
        } else {
            step(j, s);
        }
        VKMG_HIP(hipMemcpyAsync(hsum[j & 1], gsum, sizeof(double) * 8 * B, hipMemcpyDeviceToHost,
                                s));
        VKMG_HIP(hipEventRecord(ctx->step_done[j & 1], s));
        return VKMG_OK;
    };
    for (;;) {
        int nactive = 0;
        for (int k = 0; k < B; ++k) {
            Sys& q = sys[k];
            q.active = !q.done;
            q.est_last = 1.0;
            q.est_prev = 0.0;
            double* in = hinit + 8 * k;
            in[0] = q.beta0;
            in[1] = q.target;
            in[2] = q.beta;
            in[3] = q.est;
            in[4] = q.active ? 1.0 : 0.0;
            in[5] = double(q.iters);
            in[6] = double(max_iters);
            in[7] = q.active ? 1.0 / q.beta : 0.0;
            nactive += q.active;
        }
        if (nactive == 0) break;
        VKMG_HIP(hipMemcpyAsync(ginit, hinit, sizeof(double) * 8 * B, hipMemcpyHostToDevice, s));
        {
            Timed t(ctx, VKMG_KERNEL_KRYLOV, s);
            launch_givens_init(hd, HS, ginit, gsum, B, s);
            launch_scale_batched(r, n, hd + GL::kScale, HS, V, n, n, B, s);
        }
        int steps = 0;
        bool queued = false;  // step j already enqueued
        for (int j = 0; j < m; ++j) {
            if (!queued) {
                st = enqueue_step(j);
                if (st != VKMG_OK) return st;
            }
            queued = false;
            steps = j + 1;
            // pre-enqueue step j+1 unless every active system may stop at j
            if (j >= 1 && j + 1 < m) {
                bool more = false;
                for (const Sys& q : sys)
                    if (q.active && q.iters + 1 < max_iters &&
                        q.est_last * (q.est_last / q.est_prev) > 8.0 * rtol)
                        more = true;
                if (more) {
                    st = enqueue_step(j + 1);
                    if (st != VKMG_OK) return st;
                    queued = true;
                }
            }
            VKMG_HIP(hipEventSynchronize(ctx->step_done[j & 1]));
            int still = 0;
            for (int k = 0; k < B; ++k) {
                Sys& q = sys[k];
                if (!q.active) continue;
                const double* f = hsum[j & 1] + 8 * k;
                ++q.iters;
                q.est_prev = q.est_last;
                q.est_last = f[0];
                q.est = f[0];
                q.active = f[1] != 0.0;
                still += q.active;
            }
            if (still == 0) break;
        }
        // (a step enqueued past the stop runs with every system frozen; its
        // basis slot is not read, and the launches below follow it in order)
        // x += Z y per system (zero coefficients beyond its own cycle length)
        {
            Timed t(ctx, VKMG_KERNEL_KRYLOV, s);
            launch_givens_solve(hd, HS, steps, B, s);
            launch_axpy_multi(Z, S, steps, hd + GL::kY, x, n, s, B, n, HS);
        }
        // state of each system at the end of the cycle
        VKMG_HIP(hipMemcpyAsync(hsum[0], gsum, sizeof(double) * 8 * B, hipMemcpyDeviceToHost, s));
        residual();
        st = norms(r, nrm);  // synchronises the stream
        if (st != VKMG_OK) return st;
        bool all_done = true;
        for (int k = 0; k < B; ++k) {
            Sys& q = sys[k];
            const double* f = hsum[0] + 8 * k;  // estimate, active, iters, kdone, status, |g_kdone|, cycled
            if (f[6] != 0.0) {
                q.iters = int(f[2]);
                q.est = f[0];
                const double rn = nrm[k];
                q.true_rel = rn / q.beta0;
                if (f[4] != 0.0 || !std::isfinite(rn)) {
                    q.done = true;
                    q.status = VKMG_ERR_NONFINITE;
                    q.est = q.true_rel = NAN;
                } else if (rn <= q.target) {
                    q.done = true;
                    q.status = VKMG_OK;
                } else if (q.iters >= max_iters) {
                    q.done = true;
                    q.status = VKMG_ERR_NOT_CONVERGED;
                } else if (f[5] <= q.target && rn > 0.5 * q.beta) {
                    // estimate met, true residual did not and did not halve:
                    // below the rounding floor of the system
                    q.done = true;
                    q.status = VKMG_ERR_NOT_CONVERGED;
                } else {
                    q.beta = rn;
                    ++q.restarts;
                }
            }
            all_done = all_done && q.done;
        }
        if (all_done) break;
    }
    vkmg_status first = VKMG_OK;
    for (int k = 0; k < B; ++k) {
        const Sys& q = sys[k];
        if (info) {
            info[k].iterations = q.iters;
            info[k].restarts = q.restarts;
            info[k].est_rel_res = q.est;
            info[k].true_rel_res = q.true_rel;
            info[k].status = q.status;
        }
        if (first == VKMG_OK && q.status != VKMG_OK) first = q.status;
    }
    if (first == VKMG_ERR_NOT_CONVERGED)
        g_last_error = B > 1 ? "fgmres_solve: a right-hand side of the batch did not converge"
                             : "fgmres_solve: maximum iterations reached or true residual "
                               "stagnating above the tolerance";
    if (first == VKMG_ERR_NONFINITE)
        g_last_error = B > 1 ? "fgmres_solve: non-finite residual in a right-hand side of the batch"
                             : "fgmres_solve: non-finite residual";
    return first;
}

// Bytes of patch corrections one Vanka update of `level` keeps between its
// two launches: the boundary patches' (every patch's for a per-element
// viscosity), 64 slots each, per right-hand side.
size_t correction_scratch_bytes(const vkmg_ctx* c, int level) {
    const Geom& g = c->lev[level].g;
    const size_t per = c->variable ? size_t(g.N + 1) * (g.N + 1) * 64
                                   : size_t(vanka_boundary_scratch(g.N));
    return per * c->esize() * size_t(c->nb());
}

// The update half of a sweep on `level` with the patch corrections kept in
// `dbuf` (correction_scratch_bytes of device memory): x += corrections of r.
void vanka_update_with(vkmg_ctx* ctx, int level, void* x, const void* r, void* dbuf,
                       hipStream_t s) {
    LevelBuf& L = ctx->lev[level];
    const bool mfma = ctx->opt.interior_apply == VKMG_APPLY_MATRIX;
    if (ctx->variable) {
        if (ctx->opt.mg_precision == VKMG_FP64)
            launch_vanka_simple<double>(L.g, static_cast<const double*>(r), static_cast<double*>(x),
                                        static_cast<double*>(x), static_cast<const double*>(L.W),
                                        static_cast<double*>(dbuf), s, ctx->nb());
        else
            launch_vanka_simple<float>(L.g, static_cast<const float*>(r), static_cast<float*>(x),
                                       static_cast<float*>(x), static_cast<const float*>(L.W),
                                       static_cast<float*>(dbuf), s, ctx->nb());
        return;
    }
    if (ctx->opt.mg_precision == VKMG_FP64)
        launch_vanka_update<double>(L.g, static_cast<const double*>(r), static_cast<double*>(x),
                                    static_cast<double*>(x), static_cast<const double*>(L.W),
                                    static_cast<const double*>(ctx->mtab),
                                    static_cast<double*>(dbuf), ctx->opt.omega, mfma, s,
                                    ctx->nb(), parked<double>(ctx, L.g.N),
                                    ctx->tune.boundary_per_wave);
    else
        launch_vanka_update<float>(L.g, static_cast<const float*>(r), static_cast<float*>(x),
                                   static_cast<float*>(x), static_cast<const float*>(L.W),
                                   static_cast<const float*>(ctx->mtab),
                                   static_cast<float*>(dbuf), ctx->opt.omega, mfma, s,
                                   ctx->nb(), false, ctx->tune.boundary_per_wave);
}

// Launch shapes measured fastest on MI355X (profiles/ holds the autotuner
// tables they come from).  Fused sweeps are off: one workgroup then does a
// tile's residual and boundary-patch work too, which the separate launches
// spread over the whole GPU, and on the small levels, where every launch is
// latency-bound, that makes the fused launch longer than the three it
// replaces.
vkmg_tuning default_tuning(vkmg_precision p) {
    vkmg_tuning t;
    t.fused_sweep_max_n = 0;
    t.park_min_n = p == VKMG_FP64 ? 512 : std::numeric_limits<int32_t>::max();
    t.fused_prolong_max_n = 256;
    t.boundary_per_wave = 0;
    return t;
}

bool valid_tuning(const vkmg_tuning& t) {
    const int b = t.boundary_per_wave;
    return t.fused_sweep_max_n >= 0 && t.park_min_n >= 0 && t.fused_prolong_max_n >= 0 &&
           (b == 0 || b == 1 || b == 2 || b == 4 || b == 8);
}

// Median time of three runs of `reps` V-cycles (graph replays on s), in ms.
vkmg_status time_vcycles(vkmg_ctx* c, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1,
                         double* ms) {
    drop_graphs(c);
    if (!c->capture_stream) {
        hipError_t e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
        if (e != hipSuccess) return fail(VKMG_ERR_HIP, std::string("autotune stream: ") + hipGetErrorString(e));
    }
    VKMG_HIP(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
    vcycle_impl(c, c->r64, c->w64, c->capture_stream);
    hipGraph_t graph = nullptr;
    VKMG_HIP(hipStreamEndCapture(c->capture_stream, &graph));
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    VKMG_HIP(ei);
    double t[3];
    hipError_t e = hipSuccess;
    for (int w = 0; w < 2 && e == hipSuccess; ++w) e = hipGraphLaunch(exec, s);
    for (int k = 0; k < 3 && e == hipSuccess; ++k) {
        e = hipEventRecord(e0, s);
        for (int i = 0; i < reps && e == hipSuccess; ++i) e = hipGraphLaunch(exec, s);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float f = 0.0f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, e0, e1);
        t[k] = double(f) / reps;
    }
    (void)hipGraphExecDestroy(exec);
    VKMG_HIP(e);
    std::sort(t, t + 3);
    *ms = t[1];
    return VKMG_OK;
}

vkmg_status autotune_impl(vkmg_ctx* c, int reps, hipStream_t s, hipEvent_t e0, hipEvent_t e1) {
    // input: zeros (timing does not depend on the values)
    launch_fill_zero<double>(c->r64, c->top().n * c->nb(), s);
    VKMG_HIP(hipGetLastError());
    std::vector<int32_t> sizes;  // relaxed level sizes, coarse to fine
    for (int l = 1; l < c->L; ++l) sizes.push_back(c->lev[l].g.N);
    const int32_t never = std::numeric_limits<int32_t>::max();
    const bool fp64 = c->opt.mg_precision == VKMG_FP64;
    struct Knob {
        int32_t vkmg_tuning::*field;
        std::vector<int32_t> cand;
    };
    std::vector<Knob> knobs;
    {
        std::vector<int32_t> fs{0};
        for (int32_t N : sizes)
            if (N >= vanka_fused_min_n()) fs.push_back(N);
        knobs.push_back({&vkmg_tuning::fused_sweep_max_n, fs});
    }
    if (fp64) {
        std::vector<int32_t> ps(sizes.begin(), sizes.end());
        ps.push_back(never);
        knobs.push_back({&vkmg_tuning::park_min_n, ps});
        std::vector<int32_t> fp{0};
        fp.insert(fp.end(), sizes.begin(), sizes.end());
        knobs.push_back({&vkmg_tuning::fused_prolong_max_n, fp});
    }
    knobs.push_back({&vkmg_tuning::boundary_per_wave, {0, 1, 2, 4, 8}});
    double best = 0.0;
    vkmg_status st = time_vcycles(c, reps, s, e0, e1, &best);
    if (st != VKMG_OK) return st;
    for (int round = 0; round < 2; ++round) {
        for (const Knob& k : knobs) {
            const int32_t keep = c->tune.*k.field;
            int32_t choice = keep;
            for (int32_t v : k.cand) {
                if (v == keep) continue;
                c->tune.*k.field = v;
                double ms = 0.0;
                st = time_vcycles(c, reps, s, e0, e1, &ms);
                if (st != VKMG_OK) {
                    c->tune.*k.field = keep;
                    return st;
                }
                if (ms < 0.99 * best) {
                    best = ms;
                    choice = v;
                }
            }
            c->tune.*k.field = choice;
        }
    }
    drop_graphs(c);
    return VKMG_OK;
}

}  // namespace

// =====================================================================================
// C ABI
// =====================================================================================

extern "C" {

vkmg_options vkmg_default_options(void) {
    vkmg_options o;
    o.nu_pre = 2;
    o.nu_post = 2;
    o.omega = 0.5;
    o.mg_precision = VKMG_FP64;
    o.interior_apply = VKMG_APPLY_VECTOR;
    o.use_graphs = 1;
    o.batch = 1;
    o.relaxation = VKMG_RELAX_VANKA;
    o.bs_t = 1.0;
    o.bs_omega = 1.0;
    o.bs_jacobi_weight = 1.0;
    o.bs_jacobi_sweeps = 2;
    return o;
}

const char* vkmg_status_string(vkmg_status s) {
    switch (s) {
        case VKMG_OK: return "ok";
        case VKMG_ERR_INVALID_ARG: return "invalid argument";
        case VKMG_ERR_UNSUPPORTED: return "unsupported";
        case VKMG_ERR_OUT_OF_MEMORY: return "out of memory";
        case VKMG_ERR_HIP: return "HIP runtime error";
        case VKMG_ERR_SINGULAR_PATCH: return "singular patch or coarse matrix";
        case VKMG_ERR_NOT_CONVERGED: return "not converged";
        case VKMG_ERR_NONFINITE: return "non-finite value";
        case VKMG_STATUS_FORCE_INT32: break;
    }
    return "unknown status";
}

const char* vkmg_last_error(void) { return g_last_error.c_str(); }

vkmg_status vkmg_host_patch_matrix(int32_t N, double nu, double omega, int32_t cls, double* A,
                                   double* Ainv, double* Wainv, uint8_t* present) {
    if (N < 4 || cls < 0 || cls >= kClasses)
        return fail(VKMG_ERR_INVALID_ARG, "host_patch_matrix: need N >= 4 and 0 <= cls < 25");
    if (!(nu > 0.0) || !std::isfinite(nu))
        return fail(VKMG_ERR_INVALID_ARG, "host_patch_matrix: nu must be positive and finite");
    std::vector<double> Ak(kSlots * kSlots), inv;
    uint8_t pres[kSlots];
    patch_matrix(N, nu, cls, Ak.data(), pres);
    if (A) std::memcpy(A, Ak.data(), sizeof(double) * kSlots * kSlots);
    if (present) std::memcpy(present, pres, kSlots);
    std::vector<double> work = Ak;
    if (!invert_dense(kSlots, work, inv))
        return fail(VKMG_ERR_SINGULAR_PATCH, "host_patch_matrix: singular patch matrix");
    if (Ainv) std::memcpy(Ainv, inv.data(), sizeof(double) * kSlots * kSlots);
    if (Wainv) weighted_inverse(N, cls, omega, inv.data(), pres, Wainv);
    return VKMG_OK;
}

static vkmg_status setup_impl(const vkmg_grid* grid, int32_t levels, double nu,
                              const double* nu_elem, const vkmg_options* opts, void* hip_stream,
                              vkmg_ctx** out) {
    if (!grid || !out) return fail(VKMG_ERR_INVALID_ARG, "setup: NULL grid or out");
    *out = nullptr;
    if (grid->nx != grid->ny) return fail(VKMG_ERR_INVALID_ARG, "setup: nx must equal ny");
    const int N = grid->nx;
    if (levels < 2 || levels > 20) return fail(VKMG_ERR_INVALID_ARG, "setup: levels must be in [2, 20]");
    if (N < 1 || N > (1 << 15)) return fail(VKMG_ERR_INVALID_ARG, "setup: bad nx");
    if (N % (1 << (levels - 1)) != 0)
        return fail(VKMG_ERR_INVALID_ARG, "setup: nx must be divisible by 2^(levels-1)");
    const int N0 = N >> (levels - 1);
    if (N0 < 2) return fail(VKMG_ERR_INVALID_ARG, "setup: coarsest mesh must be at least 2x2");
    if (N0 > 16)
        return fail(VKMG_ERR_UNSUPPORTED,
                    "setup: coarsest mesh above 16x16 (dense coarse solve); add levels");
    if (!(nu > 0.0) || !std::isfinite(nu))
        return fail(VKMG_ERR_INVALID_ARG, "setup: nu must be positive and finite");
    vkmg_options o = opts ? *opts : vkmg_default_options();
    if (o.nu_pre < 0 || o.nu_pre > 16 || o.nu_post < 0 || o.nu_post > 16)
        return fail(VKMG_ERR_INVALID_ARG, "setup: nu_pre/nu_post must be in [0, 16]");
    if (!(o.omega > 0.0 && o.omega <= 2.0))
        return fail(VKMG_ERR_INVALID_ARG, "setup: omega must be in (0, 2]");
    if (o.mg_precision != VKMG_FP64 && o.mg_precision != VKMG_FP32)
        return fail(VKMG_ERR_INVALID_ARG, "setup: bad mg_precision");
    if (o.interior_apply != VKMG_APPLY_MATRIX && o.interior_apply != VKMG_APPLY_VECTOR)
        return fail(VKMG_ERR_INVALID_ARG, "setup: bad interior_apply");
    if (o.use_graphs != 0 && o.use_graphs != 1)
        return fail(VKMG_ERR_INVALID_ARG, "setup: use_graphs must be 0 or 1");
    if (o.batch < 1 || o.batch > 64)
        return fail(VKMG_ERR_INVALID_ARG, "setup: batch must be in [1, 64]");
    if (o.relaxation != VKMG_RELAX_VANKA && o.relaxation != VKMG_RELAX_BRAESS_SARAZIN)
        return fail(VKMG_ERR_INVALID_ARG, "setup: bad relaxation");
    if (!(o.bs_t > 0.0) || !std::isfinite(o.bs_t) || !(o.bs_omega > 0.0 && o.bs_omega <= 2.0) ||
        !(o.bs_jacobi_weight > 0.0 && o.bs_jacobi_weight <= 2.0) || o.bs_jacobi_sweeps < 1 ||
        o.bs_jacobi_sweeps > 16)
        return fail(VKMG_ERR_INVALID_ARG,
                    "setup: Braess-Sarazin parameters out of range (t > 0, omega and Jacobi "
                    "weight in (0, 2], 1..16 Jacobi sweeps)");
    // per-element viscosity: finest level as given, coarser levels by the
    // arithmetic mean of the four children
    std::vector<std::vector<double>> nul(levels);
    if (nu_elem) {
        if (o.relaxation != VKMG_RELAX_VANKA)
            return fail(VKMG_ERR_UNSUPPORTED,
                        "setup: a per-element viscosity needs Vanka relaxation");
        nul[levels - 1].assign(nu_elem, nu_elem + size_t(N) * N);
        for (double v : nul[levels - 1])
            if (!(v > 0.0) || !std::isfinite(v))
                return fail(VKMG_ERR_INVALID_ARG, "setup: viscosities must be positive and finite");
        for (int l = levels - 2; l >= 0; --l) {
            const int Nc = N >> (levels - 1 - l), Nf = 2 * Nc;
            const std::vector<double>& f = nul[l + 1];
            nul[l].resize(size_t(Nc) * Nc);
            for (int ey = 0; ey < Nc; ++ey)
                for (int ex = 0; ex < Nc; ++ex)
                    nul[l][size_t(ey) * Nc + ex] =
                        0.25 * ((f[size_t(2 * ey) * Nf + 2 * ex] + f[size_t(2 * ey) * Nf + 2 * ex + 1]) +
                                (f[size_t(2 * ey + 1) * Nf + 2 * ex] +
                                 f[size_t(2 * ey + 1) * Nf + 2 * ex + 1]));
        }
    }

    // host work first (no GPU needed to detect singular patches)
    double B1[651];
    if (!universal_interior_blocks(B1))
        return fail(VKMG_ERR_SINGULAR_PATCH, "setup: universal interior operator failed");
    std::vector<std::vector<double>> Wh(levels);
    for (int l = 1; l < levels; ++l) {
        if (nu_elem) {  // one weighted inverse per patch
            const int Nl = N >> (levels - 1 - l);
            Wh[l].resize(size_t(Nl + 1) * (Nl + 1) * kSlots * kSlots);
            if (!simple_vanka_tables(Nl, nul[l].data(), o.omega, Wh[l].data()))
                return fail(VKMG_ERR_SINGULAR_PATCH, "setup: singular Vanka patch matrix");
            continue;
        }
        const int Nl = N >> (levels - 1 - l);
        Wh[l].assign(size_t(kLevelTable), 0.0);
        for (int c = 0; c < kClasses; ++c) {
            std::vector<double> Ak(kSlots * kSlots), inv;
            uint8_t pres[kSlots];
            patch_matrix(Nl, nu, c, Ak.data(), pres);
            if (!invert_dense(kSlots, Ak, inv))
                return fail(VKMG_ERR_SINGULAR_PATCH, "setup: singular Vanka patch matrix");
            weighted_inverse(Nl, c, o.omega, inv.data(), pres, &Wh[l][size_t(c) * kSlots * kSlots]);
        }
        if (!interior_symmetry_blocks(&Wh[l][size_t(kInteriorClass) * kSlots * kSlots],
                                      &Wh[l][kDenseTable], 1e-12))
            return fail(VKMG_ERR_SINGULAR_PATCH,
                        "setup: interior patch inverse is not reflection symmetric");
        // the kernels apply the interior operator as the scaled universal one
        const double mis = universal_mismatch(&Wh[l][kDenseTable], B1, o.omega, nu, 1.0 / Nl);
        if (!(mis <= 1e-10))
            return fail(VKMG_ERR_UNSUPPORTED,
                        "setup: interior operator differs from the scaled universal form");
        // the device reads the dense inverses column by column: store W^T
        for (int c = 0; c < kClasses; ++c) {
            double* Wc = &Wh[l][size_t(c) * kSlots * kSlots];
            for (int i = 0; i < kSlots; ++i)
                for (int j = i + 1; j < kSlots; ++j) std::swap(Wc[i * kSlots + j], Wc[j * kSlots + i]);
        }
    }
    std::vector<double> Mh(kMfmaTable);
    mfma_interior_table(B1, o.mg_precision == VKMG_FP64, Mh.data());
    std::vector<float> Mf(Mh.begin(), Mh.end());
    std::vector<double> Ch;
    if (!coarse_bordered_inverse(N0, nu, Ch, nu_elem ? nul[0].data() : nullptr))
        return fail(VKMG_ERR_SINGULAR_PATCH, "setup: singular coarse matrix");

    std::unique_ptr<vkmg_ctx> c(new vkmg_ctx);
    c->L = levels;
    c->opt = o;
    c->tune = default_tuning(o.mg_precision);
    c->variable = nu_elem != nullptr;
    VKMG_HIP(hipGetDevice(&c->device));
    hipStream_t s = as_stream(hip_stream);
    c->lev.resize(levels);
    vkmg_status st = noalloc_scratch(c->device, &c->noalloc);
    const size_t es = c->esize();
    for (int l = 0; l < levels && st == VKMG_OK; ++l) {
        LevelBuf& L = c->lev[l];
        L.g = make_geom(N >> (levels - 1 - l), nu);
        const size_t nbt = size_t(o.batch);
        st = alloc(c.get(), &L.x, es * L.g.n * nbt);
        if (st == VKMG_OK) st = alloc(c.get(), &L.b, es * L.g.n * nbt);
        if (st == VKMG_OK) st = alloc(c.get(), &L.r, es * L.g.n * nbt);
        if (st == VKMG_OK && l >= 1) st = alloc(c.get(), &L.x2, es * L.g.n * nbt);
        const size_t npatch = size_t(L.g.N + 1) * (L.g.N + 1);
        if (st == VKMG_OK && l >= 1)
            st = alloc(c.get(), &L.dbuf,
                       es * (nu_elem ? npatch * 64 : size_t(vanka_boundary_scratch(L.g.N))) * nbt);
        if (st == VKMG_OK && l >= 1 && nu_elem) {
            const size_t ne = size_t(L.g.N) * L.g.N;
            st = alloc(c.get(), &L.nu, es * ne);
            if (st == VKMG_OK) {
                hipError_t e;
                if (o.mg_precision == VKMG_FP64) {
                    e = hipMemcpyAsync(L.nu, nul[l].data(), 8 * ne, hipMemcpyHostToDevice, s);
                } else {
                    std::vector<float> vf(nul[l].begin(), nul[l].end());
                    e = hipMemcpyAsync(L.nu, vf.data(), 4 * ne, hipMemcpyHostToDevice, s);
                    if (e == hipSuccess) e = hipStreamSynchronize(s);
                }
                if (e != hipSuccess) st = fail(VKMG_ERR_HIP, "setup: upload of viscosities");
            }
        }
        if (st == VKMG_OK && l >= 1 && o.relaxation == VKMG_RELAX_BRAESS_SARAZIN)
            st = alloc(c.get(), &L.bs, es * size_t(2 * L.g.nq1 + 2 * L.g.nq2) * nbt);
        if (st == VKMG_OK && l >= 1) {
            const size_t nw = nu_elem ? Wh[l].size() : size_t(kLevelTable);
            st = alloc(c.get(), &L.W, es * nw);
            if (st == VKMG_OK) {
                if (o.mg_precision == VKMG_FP64) {
                    hipError_t e = hipMemcpyAsync(L.W, Wh[l].data(), 8 * nw, hipMemcpyHostToDevice, s);
                    if (e != hipSuccess) st = fail(VKMG_ERR_HIP, "setup: upload of patch inverses");
                } else {
                    std::vector<float> wf(Wh[l].begin(), Wh[l].end());
                    hipError_t e = hipMemcpyAsync(L.W, wf.data(), 4 * nw, hipMemcpyHostToDevice, s);
                    if (e == hipSuccess) e = hipStreamSynchronize(s);
                    if (e != hipSuccess) st = fail(VKMG_ERR_HIP, "setup: upload of patch inverses");
                }
            }
        }
    }
    if (st == VKMG_OK) st = alloc(c.get(), &c->mtab, es * kMfmaTable);
    if (st == VKMG_OK) {
        const void* src = o.mg_precision == VKMG_FP64 ? static_cast<const void*>(Mh.data())
                                                      : static_cast<const void*>(Mf.data());
        hipError_t e = hipMemcpyAsync(c->mtab, src, es * kMfmaTable, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) st = fail(VKMG_ERR_HIP, "setup: upload of interior operands");
    }
    if (st == VKMG_OK) st = alloc(c.get(), reinterpret_cast<void**>(&c->C), Ch.size() * 8);
    if (st == VKMG_OK) {
        hipError_t e = hipMemcpyAsync(c->C, Ch.data(), Ch.size() * 8, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) st = fail(VKMG_ERR_HIP, "setup: upload of coarse inverse");
    }
    const int64_t n = c->top().n;
    const size_t nbt = size_t(o.batch);
    if (st == VKMG_OK && nu_elem) {
        st = alloc(c.get(), reinterpret_cast<void**>(&c->nu64), 8 * size_t(N) * N);
        if (st == VKMG_OK) {
            hipError_t e = hipMemcpyAsync(c->nu64, nul[levels - 1].data(), 8 * size_t(N) * N,
                                          hipMemcpyHostToDevice, s);
            if (e != hipSuccess) st = fail(VKMG_ERR_HIP, "setup: upload of viscosities");
        }
    }
    if (st == VKMG_OK) st = alloc(c.get(), reinterpret_cast<void**>(&c->r64), 8 * n * nbt);
    if (st == VKMG_OK) st = alloc(c.get(), reinterpret_cast<void**>(&c->w64), 8 * n * nbt);
    // partials: 264 rows of kDotBlocks, or 65 rows of dot_blocks(B) per batch entry
    if (st == VKMG_OK) {
        const size_t rows = std::max<size_t>(size_t(kDotBlocks) * 264, size_t(dot_blocks(o.batch)) * 65 * nbt);
        st = alloc(c.get(), reinterpret_cast<void**>(&c->part), 8 * rows);
    }
    if (st == VKMG_OK) st = alloc(c.get(), reinterpret_cast<void**>(&c->hdev), 8 * kHostScratch * nbt);
    if (st == VKMG_OK) {
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->hhost), 8 * kHostScratch * nbt, hipHostMallocDefault);
        if (e != hipSuccess) st = fail(VKMG_ERR_OUT_OF_MEMORY, "setup: pinned host buffer");
    }
    if (st == VKMG_OK) st = alloc(c.get(), reinterpret_cast<void**>(&c->gstat), 8 * 16 * nbt);
    if (st == VKMG_OK) {
        hipError_t e = hipHostMalloc(reinterpret_cast<void**>(&c->hstat), 8 * 24 * nbt, hipHostMallocDefault);
        if (e != hipSuccess) st = fail(VKMG_ERR_OUT_OF_MEMORY, "setup: pinned host buffer");
    }
    if (st == VKMG_OK) {
        hipError_t e = hipStreamSynchronize(s);
        if (e != hipSuccess) st = fail(VKMG_ERR_HIP, std::string("setup: ") + hipGetErrorString(e));
    }
    if (st != VKMG_OK) {
        free_all(c.get());
        return st;
    }
    *out = c.release();
    return VKMG_OK;
}

vkmg_status vkmg_setup(const vkmg_grid* grid, int32_t levels, double nu, const vkmg_options* opts,
                       void* hip_stream, vkmg_ctx** out) {
    return setup_impl(grid, levels, nu, nullptr, opts, hip_stream, out);
}

vkmg_status vkmg_setup_viscosity(const vkmg_grid* grid, int32_t levels, const double* nu_elem,
                                 const vkmg_options* opts, void* hip_stream, vkmg_ctx** out) {
    if (out) *out = nullptr;
    if (!nu_elem) return fail(VKMG_ERR_INVALID_ARG, "setup_viscosity: NULL viscosity field");
    return setup_impl(grid, levels, 1.0, nu_elem, opts, hip_stream, out);
}

void vkmg_destroy(vkmg_ctx* ctx) {
    if (!ctx) return;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    free_all(ctx);
    delete ctx;
}

vkmg_status vkmg_num_levels(const vkmg_ctx* ctx, int32_t* out) {
    if (!ctx || !out) return fail(VKMG_ERR_INVALID_ARG, "num_levels: NULL argument");
    *out = ctx->L;
    return VKMG_OK;
}

vkmg_status vkmg_layout_of(const vkmg_ctx* ctx, vkmg_layout* out) {
    if (!ctx || !out) return fail(VKMG_ERR_INVALID_ARG, "layout_of: NULL argument");
    *out = layout_of_geom(ctx->top());
    return VKMG_OK;
}

vkmg_status vkmg_level_layout(const vkmg_ctx* ctx, int32_t level, vkmg_layout* out) {
    if (!out || !check_level(ctx, level, false))
        return fail(VKMG_ERR_INVALID_ARG, "level_layout: NULL argument or level out of range");
    *out = layout_of_geom(ctx->lev[level].g);
    return VKMG_OK;
}

vkmg_status vkmg_residual(vkmg_ctx* ctx, const double* b, const double* x, double* r, void* stream) {
    if (!ctx || !b || !x || !r) return fail(VKMG_ERR_INVALID_ARG, "residual: NULL argument");
    if (r == x) return fail(VKMG_ERR_INVALID_ARG, "residual: r must not alias x");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    Timed t(ctx, VKMG_KERNEL_RESIDUAL, s);
    launch_residual<double, double>(ctx->top(), b, x, r, 0, s, ctx->nb(), ctx->nu64);
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_apply(vkmg_ctx* ctx, const double* x, double* y, void* stream) {
    if (!ctx || !x || !y) return fail(VKMG_ERR_INVALID_ARG, "apply: NULL argument");
    if (x == y) return fail(VKMG_ERR_INVALID_ARG, "apply: y must not alias x");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    Timed t(ctx, VKMG_KERNEL_RESIDUAL, s);
    launch_residual<double, double>(ctx->top(), nullptr, x, y, 1, s, ctx->nb(), ctx->nu64);
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_assemble_rhs(vkmg_ctx* ctx, const double* f, const double* g, double* b,
                              void* stream) {
    if (!ctx || !f || !b) return fail(VKMG_ERR_INVALID_ARG, "assemble_rhs: NULL f or b");
    if (b == f || b == g) return fail(VKMG_ERR_INVALID_ARG, "assemble_rhs: b must not alias f or g");
    if (ctx->variable && g)
        return fail(VKMG_ERR_UNSUPPORTED,
                    "assemble_rhs: Dirichlet data with a per-element viscosity (lift it by hand)");
    VKMG_HIP(hipSetDevice(ctx->device));
    launch_rhs(ctx->top(), f, g, b, as_stream(stream), ctx->nb());
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_assemble_rhs_adjoint(vkmg_ctx* ctx, const double* lam, double* grad_f,
                                      void* stream) {
    if (!ctx || !lam || !grad_f)
        return fail(VKMG_ERR_INVALID_ARG, "assemble_rhs_adjoint: NULL argument");
    if (static_cast<const void*>(lam) == static_cast<const void*>(grad_f))
        return fail(VKMG_ERR_INVALID_ARG, "assemble_rhs_adjoint: grad_f must not alias lam");
    VKMG_HIP(hipSetDevice(ctx->device));
    launch_rhs_adjoint(ctx->top(), lam, grad_f, as_stream(stream), ctx->nb());
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_viscosity_gradient(vkmg_ctx* ctx, const double* lam, const double* x,
                                    double* grad_nu, void* stream) {
    if (!ctx || !lam || !x || !grad_nu)
        return fail(VKMG_ERR_INVALID_ARG, "viscosity_gradient: NULL argument");
    VKMG_HIP(hipSetDevice(ctx->device));
    launch_visc_grad(ctx->top(), lam, x, grad_nu, as_stream(stream), ctx->nb());
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_remove_pressure_mean(vkmg_ctx* ctx, double* x, void* stream) {
    if (!ctx || !x) return fail(VKMG_ERR_INVALID_ARG, "remove_pressure_mean: NULL argument");
    VKMG_HIP(hipSetDevice(ctx->device));
    // scratch: the dot partials and slot 1000 of each coefficient area
    launch_pressure_mean_zero(ctx->top(), x, ctx->part, ctx->hdev + 1000, kHostScratch,
                              as_stream(stream), ctx->nb());
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_dirichlet_lift(vkmg_ctx* ctx, const double* b, double* x, void* stream) {
    if (!ctx || !b || !x) return fail(VKMG_ERR_INVALID_ARG, "dirichlet_lift: NULL argument");
    VKMG_HIP(hipSetDevice(ctx->device));
    launch_lift(ctx->top(), b, x, as_stream(stream), ctx->nb());
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_vanka_sweep(vkmg_ctx* ctx, int32_t level, void* x, const void* b, void* stream) {
    if (!x || !b || !check_level(ctx, level, true))
        return fail(VKMG_ERR_INVALID_ARG, "vanka_sweep: NULL argument or level not in [1, levels)");
    if (x == b) return fail(VKMG_ERR_INVALID_ARG, "vanka_sweep: b must not alias x");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    if (ctx->opt.mg_precision == VKMG_FP64)
        sweep_t<double>(ctx, level, static_cast<const double*>(b), static_cast<double*>(x), false, s,
                        true);
    else
        sweep_t<float>(ctx, level, static_cast<const float*>(b), static_cast<float*>(x), false, s,
                       true);
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_relax(vkmg_ctx* ctx, int32_t level, void* x, const void* b, void* stream) {
    if (!x || !b || !check_level(ctx, level, true))
        return fail(VKMG_ERR_INVALID_ARG, "relax: NULL argument or level not in [1, levels)");
    if (x == b) return fail(VKMG_ERR_INVALID_ARG, "relax: b must not alias x");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    if (ctx->opt.mg_precision == VKMG_FP64)
        sweep_t<double>(ctx, level, static_cast<const double*>(b), static_cast<double*>(x), false, s);
    else
        sweep_t<float>(ctx, level, static_cast<const float*>(b), static_cast<float*>(x), false, s);
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_vanka_update(vkmg_ctx* ctx, int32_t level, void* x, const void* r, void* stream) {
    if (!x || !r || !check_level(ctx, level, true))
        return fail(VKMG_ERR_INVALID_ARG, "vanka_update: NULL argument or level not in [1, levels)");
    if (x == r) return fail(VKMG_ERR_INVALID_ARG, "vanka_update: r must not alias x");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    Timed t(ctx, VKMG_KERNEL_VANKA, s, level);
    vanka_update_with(ctx, level, x, r, ctx->lev[level].dbuf, s);
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_vanka_update_noalloc(vkmg_ctx* ctx, int32_t level, void* x, const void* r,
                                      void* stream) {
    if (!x || !r || !check_level(ctx, level, true))
        return fail(VKMG_ERR_INVALID_ARG,
                    "vanka_update_noalloc: NULL argument or level not in [1, levels)");
    if (x == r) return fail(VKMG_ERR_INVALID_ARG, "vanka_update_noalloc: r must not alias x");
    const size_t need = correction_scratch_bytes(ctx, level);
    if (need > kNoAllocScratchBytes)
        return fail(VKMG_ERR_INVALID_ARG,
                    "vanka_update_noalloc: the patch corrections of this level need " +
                        std::to_string(need) + " bytes, more than the " +
                        std::to_string(kNoAllocScratchBytes) + "-byte static scratch");
    if (!ctx->noalloc) return fail(VKMG_ERR_HIP, "vanka_update_noalloc: no scratch address");
    VKMG_HIP(hipSetDevice(ctx->device));
    vanka_update_with(ctx, level, x, r, ctx->noalloc, as_stream(stream));
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_get_tuning(const vkmg_ctx* ctx, vkmg_tuning* out) {
    if (!ctx || !out) return fail(VKMG_ERR_INVALID_ARG, "get_tuning: NULL argument");
    *out = ctx->tune;
    return VKMG_OK;
}

vkmg_status vkmg_set_tuning(vkmg_ctx* ctx, const vkmg_tuning* tuning) {
    if (!ctx || !tuning) return fail(VKMG_ERR_INVALID_ARG, "set_tuning: NULL argument");
    if (!valid_tuning(*tuning))
        return fail(VKMG_ERR_INVALID_ARG,
                    "set_tuning: sizes must be >= 0 and boundary_per_wave 0, 1, 2, 4 or 8");
    ctx->tune = *tuning;
    drop_graphs(ctx);  // captured Arnoldi steps follow the old launch shapes
    return VKMG_OK;
}

vkmg_status vkmg_autotune(vkmg_ctx* ctx, int32_t reps, void* stream, vkmg_tuning* out) {
    if (!ctx) return fail(VKMG_ERR_INVALID_ARG, "autotune: NULL context");
    if (reps < 1) return fail(VKMG_ERR_INVALID_ARG, "autotune: reps must be >= 1");
    if (ctx->timing_mask)
        return fail(VKMG_ERR_INVALID_ARG, "autotune: kernel timing is on (vkmg_set_timing)");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    VKMG_HIP(hipEventCreate(&e0));
    hipError_t e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        (void)hipEventDestroy(e0);
        VKMG_HIP(e);
    }
    const vkmg_tuning before = ctx->tune;
    const vkmg_status st = autotune_impl(ctx, reps, s, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VKMG_OK) {
        ctx->tune = before;
        drop_graphs(ctx);
        return st;
    }
    if (out) *out = ctx->tune;
    return VKMG_OK;
}

vkmg_status vkmg_restrict(vkmg_ctx* ctx, int32_t level, const void* r_fine, void* b_coarse,
                          void* stream) {
    if (!r_fine || !b_coarse || !check_level(ctx, level, true))
        return fail(VKMG_ERR_INVALID_ARG, "restrict: NULL argument or level not in [1, levels)");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    const Geom& gf = ctx->lev[level].g;
    const Geom& gc = ctx->lev[level - 1].g;
    Timed t(ctx, VKMG_KERNEL_TRANSFER, s);
    if (ctx->opt.mg_precision == VKMG_FP64)
        launch_restrict<double>(gf, gc, static_cast<const double*>(r_fine), static_cast<double*>(b_coarse), s,
                                ctx->nb());
    else
        launch_restrict<float>(gf, gc, static_cast<const float*>(r_fine), static_cast<float*>(b_coarse), s,
                               ctx->nb());
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_prolong_add(vkmg_ctx* ctx, int32_t level, const void* e_coarse, void* x_fine,
                             void* stream) {
    if (!e_coarse || !x_fine || !check_level(ctx, level, true))
        return fail(VKMG_ERR_INVALID_ARG, "prolong_add: NULL argument or level not in [1, levels)");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    const Geom& gf = ctx->lev[level].g;
    const Geom& gc = ctx->lev[level - 1].g;
    Timed t(ctx, VKMG_KERNEL_TRANSFER, s);
    if (ctx->opt.mg_precision == VKMG_FP64)
        launch_prolong_add<double>(gf, gc, static_cast<const double*>(e_coarse), static_cast<double*>(x_fine), s,
                                   ctx->nb());
    else
        launch_prolong_add<float>(gf, gc, static_cast<const float*>(e_coarse), static_cast<float*>(x_fine), s,
                                  ctx->nb());
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_coarse_solve(vkmg_ctx* ctx, const void* r, void* e, void* stream) {
    if (!ctx || !r || !e) return fail(VKMG_ERR_INVALID_ARG, "coarse_solve: NULL argument");
    if (r == e) return fail(VKMG_ERR_INVALID_ARG, "coarse_solve: e must not alias r");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    Timed t(ctx, VKMG_KERNEL_COARSE, s);
    if (ctx->opt.mg_precision == VKMG_FP64)
        launch_coarse_gemv<double>(ctx->lev[0].g.n, ctx->C, static_cast<const double*>(r), static_cast<double*>(e), s,
                                   ctx->nb());
    else
        launch_coarse_gemv<float>(ctx->lev[0].g.n, ctx->C, static_cast<const float*>(r), static_cast<float*>(e), s,
                                  ctx->nb());
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_vcycle(vkmg_ctx* ctx, const double* r, double* z, void* stream) {
    if (!ctx || !r || !z) return fail(VKMG_ERR_INVALID_ARG, "vcycle: NULL argument");
    if (r == z) return fail(VKMG_ERR_INVALID_ARG, "vcycle: z must not alias r");
    VKMG_HIP(hipSetDevice(ctx->device));
    vcycle_impl(ctx, r, z, as_stream(stream));
    VKMG_HIP(hipGetLastError());
    return VKMG_OK;
}

vkmg_status vkmg_fgmres_solve(vkmg_ctx* ctx, const double* b, double* x, double rtol,
                              int32_t restart, int32_t max_iters, vkmg_info* info, void* stream) {
    if (info) {
        const int nbi = ctx ? ctx->nb() : 1;
        std::memset(info, 0, sizeof(*info) * size_t(nbi));
        for (int k = 0; k < nbi; ++k) info[k].status = VKMG_ERR_INVALID_ARG;
    }
    if (!ctx || !b || !x) return fail(VKMG_ERR_INVALID_ARG, "fgmres_solve: NULL argument");
    if (b == x) return fail(VKMG_ERR_INVALID_ARG, "fgmres_solve: x must not alias b");
    if (restart < 1 || restart > 256) return fail(VKMG_ERR_INVALID_ARG, "fgmres_solve: restart must be in [1, 256]");
    if (max_iters < 1) return fail(VKMG_ERR_INVALID_ARG, "fgmres_solve: max_iters must be >= 1");
    if (!(rtol >= 0.0) || !std::isfinite(rtol)) return fail(VKMG_ERR_INVALID_ARG, "fgmres_solve: bad rtol");
    if (ctx->nb() > 1 && restart > kDelayedMaxRestart)
        return fail(VKMG_ERR_UNSUPPORTED, "fgmres_solve: batched contexts need restart <= 32");
    VKMG_HIP(hipSetDevice(ctx->device));
    hipStream_t s = as_stream(stream);
    vkmg_status st = ensure_basis(ctx, restart);
    if (st != VKMG_OK) return st;
    if (restart <= kDelayedMaxRestart)
        return fgmres_delayed(ctx, b, x, rtol, restart, max_iters, info, s);
    const Geom& g = ctx->top();
    const int64_t n = g.n;
    const int64_t ld = basis_stride(n);
    const int m = restart;
    double* r = ctx->r64;
    double* w = ctx->w64;
    double* V = ctx->V;
    double* Z = ctx->Z;

    auto residual = [&](void) {
        Timed t(ctx, VKMG_KERNEL_RESIDUAL, s);
        launch_residual<double, double>(g, b, x, r, 0, s, 1, ctx->nu64);
    };
    residual();
    double beta0 = 0.0;
    st = norm_sync(ctx, r, &beta0, s);
    if (st != VKMG_OK) return st;
    auto finish = [&](vkmg_status status, int it, int rs, double est, double tru) {
        if (info) {
            info->iterations = it;
            info->restarts = rs;
            info->est_rel_res = est;
            info->true_rel_res = tru;
            info->status = status;
        }
        if (status == VKMG_ERR_NOT_CONVERGED)
            g_last_error = "fgmres_solve: maximum iterations reached above the tolerance";
        if (status == VKMG_ERR_NONFINITE) g_last_error = "fgmres_solve: non-finite residual";
        return status;
    };
    if (!std::isfinite(beta0)) return finish(VKMG_ERR_NONFINITE, 0, 0, NAN, NAN);
    if (beta0 == 0.0) return finish(VKMG_OK, 0, 0, 0.0, 0.0);
    const double target = rtol * beta0;
    int total = 0, restarts = 0;
    double beta = beta0;
    // Hu: the Hessenberg matrix as built; R: its columns after the Givens
    // rotations; gbase: the right-hand side beta e1 after the rotations of
    // the columns before the previous one (the same bookkeeping as the
    // device Givens kernel of the delayed scheme, where that column is
    // finalised one step late; here redoing its rotation changes nothing)
    std::vector<double> Hu(size_t(m + 1) * m), R(size_t(m + 1) * m), cs(m), sn(m), gbase(m + 1),
        gv(m + 1), y(m);
    auto Hij = [&](int i, int j) -> double& { return Hu[size_t(i) * m + j]; };
    auto Rij = [&](int i, int j) -> double& { return R[size_t(i) * m + j]; };
    auto rotate_column = [&](int j) {
        for (int i = 0; i <= j + 1; ++i) Rij(i, j) = Hij(i, j);
        for (int i = 0; i < j; ++i) {
            const double t = cs[i] * Rij(i, j) + sn[i] * Rij(i + 1, j);
            Rij(i + 1, j) = -sn[i] * Rij(i, j) + cs[i] * Rij(i + 1, j);
            Rij(i, j) = t;
        }
        const double denom = std::hypot(Rij(j, j), Rij(j + 1, j));
        cs[j] = Rij(j, j) / denom;
        sn[j] = Rij(j + 1, j) / denom;
        Rij(j, j) = denom;
        Rij(j + 1, j) = 0.0;
    };
    auto rotate_rhs = [&](std::vector<double>& g, int j) {
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
    };
    double est = 1.0;
    double* h1 = ctx->hdev;        // first Gram-Schmidt pass, j+1 values
    double* h2 = ctx->hdev + 300;  // second pass, j+1 values, then ||w||^2 at [j+1]
    // Restarts > 32 (shorter ones take fgmres_delayed): classical
    // Gram-Schmidt with one reorthogonalisation (Giraud et al.'s CGS2,
    // orthogonal to working accuracy; multi-vector passes): h1 = V^T w;
    // w' = w - V h1 with h2 = V^T w' and |w'|^2 in the same pass;
    // v_{j+1} = (w' - V h2) / |w' - V h2| in a third, with
    // |w' - V h2|^2 = |w'|^2 - |h2|^2 (V orthonormal).  Beyond 32 basis
    // vectors: unfused passes, |w''|^2 into h2[kb], v_{j+1} scaled on host
    // request.
    // Every pointer depends only on j, so a step can be captured once per j
    // and replayed.
    const bool fp32_mg = ctx->opt.mg_precision == VKMG_FP32;
    auto arnoldi_step = [&](int j, hipStream_t ss) {
        double* vj = V + int64_t(j) * ld;
        double* zj = Z + int64_t(j) * ld;
        const int kb = j + 1;
        // FP32 multigrid: z_j stays FP32 and the apply w = A z_j writes it
        // widened into the basis
        vcycle_impl(ctx, vj, zj, ss, false, fp32_mg);
        {
            Timed t(ctx, VKMG_KERNEL_RESIDUAL, ss);
            if (fp32_mg)
                launch_apply_widen(g, static_cast<const float*>(ctx->lev.back().x), w, zj, ss,
                                   ctx->nu64);
            else
                launch_residual<double, double>(g, nullptr, zj, w, 1, ss, 1, ctx->nu64);
        }
        dots_async(ctx, V, ld, kb, w, h1, ss);
        if (kb <= 32) {
            Timed t(ctx, VKMG_KERNEL_KRYLOV, ss);
            launch_update_dot(V, ld, kb, h1, w, n, ctx->part, ss);
            launch_reduce_partials(ctx->part, kb + 1, h2, ss);
            launch_normalize(V, ld, kb, h2, h2 + kb, w, V + int64_t(kb) * ld, n, ss);
        } else {
            {
                Timed t(ctx, VKMG_KERNEL_KRYLOV, ss);
                launch_update(V, ld, kb, h1, w, n, ss);
            }
            dots_async(ctx, V, ld, kb, w, h2, ss);
            {
                Timed t(ctx, VKMG_KERNEL_KRYLOV, ss);
                launch_update(V, ld, kb, h2, w, n, ss);
            }
            dots_async(ctx, w, 0, 1, w, h2 + kb, ss);
        }
    };
    // graphs replace the ~100 launches of a step by one; bypassed while
    // kernels are timed (events recorded inside a replayed graph cannot be
    // read back with hipEventElapsedTime)
    const bool use_graphs = ctx->opt.use_graphs != 0 && ctx->timing_mask == 0;
    if (use_graphs && ctx->graphs_scheme != 0) {
        drop_graphs(ctx);
        ctx->graphs_scheme = 0;
    }
    auto enqueue_step = [&](int j) -> vkmg_status {
        if (use_graphs) {
            vkmg_status sg = step_graph(ctx, j, arnoldi_step);
            if (sg != VKMG_OK) return sg;
            VKMG_HIP(hipGraphLaunch(ctx->step_graphs[j], s));
        } else {
            arnoldi_step(j, s);
        }
        return VKMG_OK;
    };
    for (;;) {
        {
            Timed t(ctx, VKMG_KERNEL_KRYLOV, s);
            launch_scale(r, 1.0 / beta, V, n, s);
        }
        std::fill(Hu.begin(), Hu.end(), 0.0);
        std::fill(gbase.begin(), gbase.end(), 0.0);
        gbase[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            const int kb = j + 1;  // basis vectors so far
            const bool normalized = kb <= 32;
            double hnext = 0.0;
            st = enqueue_step(j);
            if (st != VKMG_OK) return st;
            bool finite = true;
            VKMG_HIP(hipMemcpyAsync(ctx->hhost, h1, sizeof(double) * kb, hipMemcpyDeviceToHost, s));
            VKMG_HIP(hipMemcpyAsync(ctx->hhost + 300, h2, sizeof(double) * (kb + 1), hipMemcpyDeviceToHost, s));
            VKMG_HIP(hipStreamSynchronize(s));
            double hh = 0.0;
            for (int i = 0; i <= j; ++i) {
                Hij(i, j) = ctx->hhost[i] + ctx->hhost[300 + i];
                hh += ctx->hhost[300 + i] * ctx->hhost[300 + i];
            }
            if (normalized) {
                // the formula of the normalisation kernel
                const double d = ctx->hhost[300 + kb] - hh;
                hnext = d > 0.0 ? std::sqrt(d) : 0.0;
            } else {
                hnext = std::sqrt(ctx->hhost[300 + kb]);
            }
            for (int i = 0; i <= j; ++i) finite = finite && std::isfinite(Hij(i, j));
            Hij(j + 1, j) = hnext;
            if (!finite || !std::isfinite(hnext))
                return finish(VKMG_ERR_NONFINITE, total, restarts, NAN, NAN);
            if (j > 0) {
                rotate_column(j - 1);
                rotate_rhs(gbase, j - 1);
            }
            rotate_column(j);
            gv = gbase;
            rotate_rhs(gv, j);
            const bool breakdown = hnext == 0.0;
            if (!breakdown && !normalized) {
                Timed t(ctx, VKMG_KERNEL_KRYLOV, s);
                launch_scale(w, 1.0 / hnext, V + int64_t(j + 1) * ld, n, s);
            }
            ++total;
            k = j + 1;
            est = std::fabs(gv[j + 1]) / beta0;
            if (std::fabs(gv[j + 1]) <= target) break;
            if (breakdown || total >= max_iters) break;
        }
        // y = H^{-1} g (upper triangular)
        for (int i = k - 1; i >= 0; --i) {
            double acc = gv[i];
            for (int l = i + 1; l < k; ++l) acc -= Rij(i, l) * y[l];
            y[i] = acc / Rij(i, i);
        }
        std::memcpy(ctx->hhost + 600, y.data(), sizeof(double) * k);
        VKMG_HIP(hipMemcpyAsync(ctx->hdev + 600, ctx->hhost + 600, sizeof(double) * k, hipMemcpyHostToDevice, s));
        {
            Timed t(ctx, VKMG_KERNEL_KRYLOV, s);
            launch_axpy_multi(Z, ld, k, ctx->hdev + 600, x, n, s);
        }
        residual();
        double rn = 0.0;
        st = norm_sync(ctx, r, &rn, s);
        if (st != VKMG_OK) return st;
        if (!std::isfinite(rn)) return finish(VKMG_ERR_NONFINITE, total, restarts, est, NAN);
        if (rn <= target) return finish(VKMG_OK, total, restarts, est, rn / beta0);
        if (total >= max_iters) return finish(VKMG_ERR_NOT_CONVERGED, total, restarts, est, rn / beta0);
        // the Arnoldi estimate met the tolerance but the true residual did
        // not, and the cycle did not halve it: the tolerance is below what
        // FP64 residuals of this system can resolve; more cycles only repeat
        if (std::fabs(gv[k]) <= target && rn > 0.5 * beta) {
            finish(VKMG_ERR_NOT_CONVERGED, total, restarts, est, rn / beta0);
            g_last_error = "fgmres_solve: true residual stagnates above the tolerance (rounding floor)";
            return VKMG_ERR_NOT_CONVERGED;
        }
        ++restarts;
        beta = rn;
    }
}

vkmg_status vkmg_set_timing(vkmg_ctx* ctx, int32_t class_mask) {
    if (!ctx) return fail(VKMG_ERR_INVALID_ARG, "set_timing: NULL context");
    VKMG_HIP(hipSetDevice(ctx->device));
    for (int k = 0; k < VKMG_KERNEL_COUNT; ++k) {
        for (auto& e : ctx->events[k]) {
            (void)hipEventSynchronize(e.stop);
            (void)hipEventDestroy(e.start);
            (void)hipEventDestroy(e.stop);
        }
        ctx->events[k].clear();
    }
    ctx->timing_mask = class_mask;
    return VKMG_OK;
}

vkmg_status vkmg_kernel_timing(vkmg_ctx* ctx, int32_t kernel_class, int32_t level,
                               int64_t* launches, double* total_ms) {
    if (!ctx || kernel_class < 0 || kernel_class >= VKMG_KERNEL_COUNT)
        return fail(VKMG_ERR_INVALID_ARG, "kernel_timing: bad context or class");
    if (level < -1 || level >= ctx->L)
        return fail(VKMG_ERR_INVALID_ARG, "kernel_timing: level must be -1 or in [0, levels)");
    VKMG_HIP(hipSetDevice(ctx->device));
    int64_t n = 0;
    double ms_sum = 0.0;
    for (auto& e : ctx->events[kernel_class]) {
        if (level != -1 && e.level != level) continue;
        VKMG_HIP(hipEventSynchronize(e.stop));
        float ms = 0.f;
        VKMG_HIP(hipEventElapsedTime(&ms, e.start, e.stop));
        ms_sum += ms;
        ++n;
    }
    if (launches) *launches = n;
    if (total_ms) *total_ms = ms_sum;
    return VKMG_OK;
}

}  // extern "C"
