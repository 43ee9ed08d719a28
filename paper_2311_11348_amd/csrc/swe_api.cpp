// Host runtime behind the C ABI declared in include/swe_dg.h.
//
// It validates and preprocesses the mesh (connectivity from shared vertex
// pairs, boundary codes, Morton ordering of elements by centroid and of
// vertices by first use, so that neighbour gathers stay in cache), owns the
// device buffers and streams, converts between the caller's physical
// orthonormal coefficients [elem][comp][mode] and the device's
// reference-scaled structure-of-arrays layout, and enqueues the stage kernels.
#include "../../include/swe_dg.h"
#include "swe_internal.h"
#include "swe_tables.h"

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <sched.h>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

using namespace swe;

namespace {

constexpr int K_OF[4] = {1, 3, 6, 10};
constexpr double QX[SWET_NQP] = SWET_QX;
constexpr double QY[SWET_NQP] = SWET_QY;
constexpr double QW[SWET_NQP] = SWET_QW;
constexpr double QPHI[SWET_NQP][10] = SWET_QPHI;

}  // namespace

struct swe_ctx {
    swe_config cfg{};
    bool fp32 = false;
    int K = 1;
    size_t rsz = 8;
    int64_t ne = 0, nv = 0;
    int stride = 0;
    bool have_mesh = false;
    std::vector<int> e_perm, e_iperm;     // internal -> user, user -> internal
    std::vector<int> v_perm, v_iperm;
    std::vector<double> vx, vy, hb;       // internal vertex order
    std::vector<int> ev;                  // [3][stride]
    std::vector<double> sfac;             // sqrt(|det B_e|), internal order
    std::vector<signed char> p;           // internal order
    bool uniform = true;
    double4 *d_vtx = nullptr;
    int *d_ev = nullptr, *d_nb = nullptr;
    unsigned char *d_nbk = nullptr;
    signed char *d_p = nullptr;
    void *d_C[2] = {nullptr, nullptr}, *d_U[2] = {nullptr, nullptr};
    void *d_L = nullptr, *d_src = nullptr;
    int *d_flag = nullptr;
    double *d_part = nullptr, *d_mass = nullptr;
    // order-separated scheme: elements with a correction, grouped by order
    unsigned char *d_inlist = nullptr;
    signed char *d_pnew = nullptr;
    double *d_I = nullptr;
    void *d_Lb = nullptr, *d_Lc = nullptr;
    int *d_list = nullptr, *d_cnt = nullptr;
    int list_off[5] = {0, 0, 0, 0, 0};
    int list_cnt[4] = {0, 0, 0, 0};
    std::vector<int> nb_host;             // [3][stride] neighbour ids / boundary codes
    std::vector<unsigned char> nbk_host;  // [stride] neighbours' local edge ids, 2 bits per edge
    // static order map of a separated context: elements renumbered so that
    // the unlisted ones come first and each order's listed ones follow in
    // one contiguous range (each group in Morton order)
    bool grouped = false;
    int64_t n_unlisted = 0;
    int64_t halo_start = 0;               // separated grouping: first unlisted neighbour of a listed element
    // heterogeneous stages: pinned host copies of the stage input state and
    // of the correction, and the vertices in the device's layout
    void *h_C = nullptr, *h_U = nullptr, *h_Lc = nullptr;
    std::vector<double4> h_vtx;
    hipEvent_t ev_ready = nullptr, ev_corr = nullptr;
    swe_batch *batch = nullptr;           // resident in this batch, or null
    int slot = -1;
    hipStream_t s_base = nullptr, s_corr = nullptr;
    bool own_base = false, own_corr = false;
    double t = 0.0;
    bool failed = false;
    int ncon = 0;
    double amp[NCON_MAX] = {0}, omega[NCON_MAX] = {0}, phase[NCON_MAX] = {0};
    // replayed step: one graph per step, clock (time, forcing) on the device
    unsigned *d_items = nullptr;           // edge items of the shared-flux stage kernel, per block
    int *d_item_off = nullptr;            // [blocks + 1]
    int64_t item_blocks = 0;              // the leading blocks whose items are built
    InstDesc *d_inst = nullptr;
    hipGraph_t step_graph = nullptr, multi_graph = nullptr;   // one step; GRAPH_STEPS steps
    hipGraphExec_t step_exec = nullptr, multi_exec = nullptr;
    std::vector<long long> graph_key;     // what the step graph was built for
    std::string err;
};

namespace {

swe_status fail(swe_ctx *c, swe_status s, const std::string &msg)
{
    if (c) c->err = msg;
    return s;
}

#define HIP_TRY(ctx, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return fail((ctx), e_ == hipErrorOutOfMemory ? SWE_ENOMEM : SWE_EDEVICE,              \
                        std::string(#expr) + ": " + hipGetErrorString(e_));                      \
    } while (0)

// Every transfer of a context is ordered on its base stream (the library's
// kernels run on non-blocking streams, which the null stream does not order
// against); host-to-device copies wait until the data has left the host
// buffer, device-to-host copies first wait for the context's queued work.
hipError_t h2d(swe_ctx *c, void *dst, const void *src, size_t bytes)
{
    hipError_t e = hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->s_base);
    return e == hipSuccess ? hipStreamSynchronize(c->s_base) : e;
}

hipError_t d2h(swe_ctx *c, void *dst, const void *src, size_t bytes)
{
    hipError_t e = hipStreamSynchronize(c->s_corr);
    if (e == hipSuccess) e = hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->s_base);
    return e == hipSuccess ? hipStreamSynchronize(c->s_base) : e;
}

hipError_t dzero(swe_ctx *c, void *dst, size_t bytes) { return hipMemsetAsync(dst, 0, bytes, c->s_base); }

void drop_step_graph(swe_ctx *c)
{
    if (c->step_exec) (void)hipGraphExecDestroy(c->step_exec);
    if (c->step_graph) (void)hipGraphDestroy(c->step_graph);
    if (c->multi_exec) (void)hipGraphExecDestroy(c->multi_exec);
    if (c->multi_graph) (void)hipGraphDestroy(c->multi_graph);
    c->step_exec = c->multi_exec = nullptr;
    c->step_graph = c->multi_graph = nullptr;
    c->graph_key.clear();
}

void free_mesh(swe_ctx *c)
{
    drop_step_graph(c);
    if (c->d_inst) (void)hipFree(c->d_inst);
    c->d_inst = nullptr;
    if (c->d_items) (void)hipFree(c->d_items);
    if (c->d_item_off) (void)hipFree(c->d_item_off);
    c->d_items = nullptr;
    c->d_item_off = nullptr;
    void *ptrs[] = {c->d_vtx, c->d_ev, c->d_nb, c->d_nbk, c->d_p, c->d_C[0], c->d_C[1],
                    c->d_U[0], c->d_U[1], c->d_L, c->d_src, c->d_flag, c->d_part, c->d_mass,
                    c->d_inlist, c->d_Lb, c->d_Lc, c->d_list, c->d_cnt, c->d_pnew, c->d_I};
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    c->d_vtx = nullptr; c->d_ev = nullptr; c->d_nb = nullptr; c->d_nbk = nullptr; c->d_p = nullptr;
    c->d_C[0] = c->d_C[1] = c->d_U[0] = c->d_U[1] = nullptr;
    c->d_L = c->d_src = nullptr;
    c->d_flag = nullptr; c->d_part = nullptr; c->d_mass = nullptr;
    c->d_inlist = nullptr; c->d_Lb = nullptr; c->d_Lc = nullptr; c->d_list = nullptr; c->d_cnt = nullptr;
    c->d_pnew = nullptr; c->d_I = nullptr;
    void *h[] = {c->h_C, c->h_U, c->h_Lc};
    for (void *q : h)
        if (q) (void)hipHostFree(q);
    c->h_C = c->h_U = c->h_Lc = nullptr;
    c->h_vtx.clear();
    c->have_mesh = false;
}

// A batch member's state buffers (C0, C1, U0, U1, the right-hand-side
// scratch, edge items) are released while it is resident: its state lives in
// the batch's pool.  They are re-created (zero-filled) when the state comes
// back; the edge items when the member leaves the batch.
void release_state_buffers(swe_ctx *c)
{
    drop_step_graph(c);
    void *q[] = {c->d_C[0], c->d_C[1], c->d_U[0], c->d_U[1], c->d_L, c->d_items, c->d_item_off};
    for (void *x : q)
        if (x) (void)hipFree(x);
    c->d_C[0] = c->d_C[1] = c->d_U[0] = c->d_U[1] = c->d_L = nullptr;
    c->d_items = nullptr;
    c->d_item_off = nullptr;
    c->item_blocks = 0;
}

swe_status restore_state_buffers(swe_ctx *c)
{
    if (c->d_C[0]) return SWE_OK;
    const size_t w = c->rsz, K = c->K, S = c->stride;
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(c, hipMalloc(&c->d_C[b], w * 3 * K * S));
        HIP_TRY(c, hipMalloc(&c->d_U[b], w * 2 * K * S));
        HIP_TRY(c, dzero(c, c->d_C[b], w * 3 * K * S));
        HIP_TRY(c, dzero(c, c->d_U[b], w * 2 * K * S));
    }
    HIP_TRY(c, hipMalloc(&c->d_L, w * 3 * K * S));
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    return SWE_OK;
}

double xi_hat(const swe_ctx *c, double t)
{
    double s = 0.0;
    for (int i = 0; i < c->ncon; ++i) s += c->amp[i] * std::sin(c->omega[i] * t + c->phase[i]);
    return s;
}

uint32_t spread16(uint32_t x)
{
    x &= 0xffff;
    x = (x | (x << 8)) & 0x00ff00ff;
    x = (x | (x << 4)) & 0x0f0f0f0f;
    x = (x | (x << 2)) & 0x33333333;
    x = (x | (x << 1)) & 0x55555555;
    return x;
}

MeshView view(const swe_ctx *c)
{
    MeshView m;
    m.ne = (int)c->ne;
    m.stride = c->stride;
    m.KS = c->K;
    m.vtx = c->d_vtx;
    m.ev = c->d_ev;
    m.enb = c->d_nb;
    m.enbk = c->d_nbk;
    m.ep = c->d_p;
    return m;
}

// the edge items cover the first nblocks blocks (0: every block)
bool items_cover(const swe_ctx *c, int64_t nblocks);

template <typename Real>
StageArgs<Real> make_args(const swe_ctx *c)
{
    StageArgs<Real> a;
    std::memset(&a, 0, sizeof(a));
    a.m = view(c);
    a.ph.g = c->cfg.g;
    a.ph.fc = c->cfg.f_coriolis;
    a.ph.fric = c->cfg.friction_coef;
    a.ph.friction = c->cfg.friction;
    a.flag = c->d_flag;
    a.mixed = c->uniform ? 0 : 1;
    a.src = static_cast<const Real *>(c->d_src);
    return a;
}

// Where the kernels of a step go: the context's two streams joined by
// events, or two branches of a step graph under construction (graph set).
// A step graph whose orders are re-chosen on the device is one chain (the
// list kernels after the base pass of the same stage): its lists are short,
// and a fork and a join cost more than the list kernel's own time (measured
// on the adaptive tsunami; the static maps of the dam break keep the two
// branches, where they overlap long lists with the base pass).
struct Lanes {
    swe_ctx *c;
    Sink a, b;           // base work, correction work
    bool graph = false, chain = false;
    explicit Lanes(swe_ctx *cc) : c(cc)
    {
        a.s = c->s_base;
        b.s = c->s_corr;
    }
    Lanes(swe_ctx *cc, hipGraph_t g) : c(cc), graph(true), chain(cc->cfg.adapt != 0)
    {
        a.g = g;
        b.g = g;
    }
    // where the correction (list) work goes
    Sink &side() { return chain ? a : b; }
    // the correction branch starts after everything enqueued on the base branch so far
    hipError_t fork()
    {
        if (chain) return hipSuccess;
        if (graph) {
            b.ndep = a.ndep;
            for (int i = 0; i < Sink::MAXDEP; ++i) b.dep[i] = a.dep[i];
            return hipSuccess;
        }
        const hipError_t e = hipEventRecord(c->ev_ready, c->s_base);
        return e == hipSuccess ? hipStreamWaitEvent(c->s_corr, c->ev_ready, 0) : e;
    }
    // base work enqueued next waits for the correction branch
    hipError_t join()
    {
        if (chain) return hipSuccess;
        if (graph) return a.join(b) ? hipSuccess : hipErrorInvalidValue;
        const hipError_t e = hipEventRecord(c->ev_corr, c->s_corr);
        return e == hipSuccess ? hipStreamWaitEvent(c->s_base, c->ev_corr, 0) : e;
    }

    // stage time: from the host, or (graph) from the device clock of the step
    template <typename Real>
    void time(StageArgs<Real> &args, int stage, double t, double dt) const
    {
        if (graph) {
            args.inst = c->d_inst;
            args.stage = stage;
        } else {
            args.xihat = xi_hat(c, t);
            args.dt = dt;
        }
    }
};

// launch one stage; in/out buffer indices follow the Shu-Osher form
template <typename Real>
hipError_t enqueue_stage(Lanes &L, int mode, int in, int out, double tstage, double dt, const void *Cn,
                         void *Lout)
{
    swe_ctx *c = L.c;
    StageArgs<Real> a = make_args<Real>(c);
    a.Cin = static_cast<const Real *>(c->d_C[in]);
    a.Uin = static_cast<const Real *>(c->d_U[in]);
    a.Cn = static_cast<const Real *>(Cn);
    a.Cout = out >= 0 ? static_cast<Real *>(c->d_C[out]) : nullptr;
    a.Uout = out >= 0 ? static_cast<Real *>(c->d_U[out]) : nullptr;
    a.Lout = static_cast<Real *>(Lout);
    L.time(a, mode == MODE_STAGE2 ? 1 : 0, tstage, dt);
    if (items_cover(c, 0) && !a.mixed)
        return launch_stage_sh(c->cfg.p_max, c->fp32, mode, &a, c->d_items, c->d_item_off, L.a);
    return launch_stage(c->cfg.p_max, c->fp32, mode, false, &a, L.a);
}

template <typename Real>
hipError_t enqueue_stage(swe_ctx *c, int mode, int in, int out, double tstage, double dt, const void *Cn,
                         void *Lout)
{
    Lanes L(c);
    return enqueue_stage<Real>(L, mode, in, out, tstage, dt, Cn, Lout);
}

bool separated(const swe_ctx *c) { return c->cfg.separate && c->cfg.p_base < c->cfg.p_max; }

// Base pass of the order-separated and order-partitioned schemes over the
// elements [0, end): the shared-flux kernel at the base order (orders 1..3)
// on the leading blocks that have edge items, the element-gather kernel on
// the rest of the range (all of it without items).
template <typename Real>
hipError_t launch_base(Lanes &L, int mode, StageArgs<Real> &a, int64_t end)
{
    swe_ctx *c = L.c;
    const int b = c->cfg.p_base;
    const int64_t all = (c->ne + BLOCK - 1) / BLOCK, nb_end = (end + BLOCK - 1) / BLOCK;
    const int64_t cov = (c->d_items && stage_sh_supported(b, c->fp32)) ? std::min(c->item_blocks, nb_end) : 0;
    hipError_t e = hipSuccess;
    if (cov > 0) {
        a.blocks = cov < all ? (int)cov : 0;
        e = launch_stage_sh(b, c->fp32, mode, &a, c->d_items, c->d_item_off, L.a);
        a.blocks = 0;
        if (e != hipSuccess) return e;
    }
    const int64_t off = cov * BLOCK;
    if (off < end) {
        StageArgs<Real> r = a;
        r.e_off = (int)off;
        r.m.ne = (int)(end - off);
        e = launch_stage(b, c->fp32, mode, true, &r, L.a);
    }
    return e;
}

// Blocks per order of a one-launch list kernel (every order's list fits):
// with adaptivity the lengths live on the device and each may reach ne.
int list_blocks(const swe_ctx *c)
{
    if (c->cfg.adapt) return (int)((c->ne + BLOCK - 1) / BLOCK);
    int most = 0;
    for (int p = c->cfg.p_base; p <= c->cfg.p_max; ++p) most = std::max(most, c->list_cnt[p]);
    return (most + BLOCK - 1) / BLOCK;
}


// Order adaptation at the start of a step, from the state in buffer 0.
template <typename Real>
hipError_t enqueue_adapt(Lanes &L, double tn)
{
    swe_ctx *c = L.c;
    StageArgs<Real> a = make_args<Real>(c);
    a.Cin = static_cast<const Real *>(c->d_C[0]);
    L.time(a, 0, tn, 0.0);
    a.cntw = c->d_cnt;
    hipError_t e = launch_indicator(c->fp32, &a, c->cfg.adapt_tau, c->cfg.p_base, c->cfg.p_max, nullptr,
                                    c->d_pnew, L.a);
    if (e != hipSuccess) return e;
    a.Cout = static_cast<Real *>(c->d_C[0]);
    a.Calt = static_cast<Real *>(c->d_C[1]);
    a.Uout = static_cast<Real *>(c->d_U[0]);
    a.Ualt = static_cast<Real *>(c->d_U[1]);
    a.inlist = c->d_inlist;
    a.listw = c->d_list;
    // a step graph advances its clock here, after the indicator read the step's start time
    return launch_apply_order(c->cfg.p_max, c->fp32, &a, c->d_pnew, c->d_p, c->cfg.p_base, (int)c->ne,
                              L.graph ? c->d_inst : nullptr, c->d_flag, L.a);
}

// Order-separated stage: base kernel over all elements (branch A) while the
// corrections of the listed elements run on branch B; the epilogue of the
// listed elements joins both on branch A.  In one chain (adaptive step
// graphs) the corrections follow the base pass and do the join themselves.
template <typename Real>
hipError_t enqueue_separated(Lanes &L, int mode, int in, int out, double tstage, double dt)
{
    swe_ctx *c = L.c;
    const int b = c->cfg.p_base, pm = c->cfg.p_max;
    StageArgs<Real> a = make_args<Real>(c);
    a.mixed = 0;
    a.Cin = static_cast<const Real *>(c->d_C[in]);
    a.Uin = static_cast<const Real *>(c->d_U[in]);
    a.Cn = static_cast<const Real *>(c->d_C[0]);
    a.Cout = static_cast<Real *>(c->d_C[out]);
    a.Uout = static_cast<Real *>(c->d_U[out]);
    L.time(a, mode == MODE_STAGE2 ? 1 : 0, tstage, dt);
    a.inlist = c->d_inlist;
    a.Lb = static_cast<Real *>(c->d_Lb);
    a.Lc = static_cast<Real *>(c->d_Lc);
    hipError_t e = L.fork();
    if (e != hipSuccess) return e;
    // every element: a listed one leaves its base part in Lb for the epilogue
    e = launch_base<Real>(L, mode, a, c->ne);
    if (e != hipSuccess) return e;
    // the corrections of every order in one launch on branch B, then (after
    // the join) the epilogues of every order in one launch
    a.list = c->d_list;
    a.count = c->d_cnt;
    const int nblk = list_blocks(c), lcap = (int)c->ne;
    // one chain: the corrections run after the base pass, so they join the
    // base parts and finish the listed elements' stage themselves (the sum
    // the epilogue would form, bit for bit), one dependent launch less
    if (L.chain) a.finish = mode;
    e = launch_corr_all(b, pm, c->fp32, &a, dt, nblk, lcap, L.side());
    if (e != hipSuccess || L.chain) return e;
    e = L.join();
    if (e != hipSuccess) return e;
    return launch_epi_all(b, pm, c->fp32, mode, &a, nblk, lcap, L.a);
}

// Heterogeneous order-separated stage (a static order map in the separated
// grouping: unlisted elements, their neighbours of listed elements, then the
// listed elements of each order).  The GPU runs the base pass over every
// element; meanwhile the stage's input state of the neighbour and listed
// ranges comes down to the host, whose threads compute the listed elements'
// correction with the GPU's element code; the correction goes back up and
// the epilogue joins it on the GPU.
template <typename Real>
hipError_t host_mirrors(swe_ctx *c)
{
    if (c->h_C) return hipSuccess;
    const size_t S = c->stride, K = c->K;
    hipError_t e = hipHostMalloc(&c->h_C, sizeof(Real) * 3 * K * S, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&c->h_U, sizeof(Real) * 2 * K * S, hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc(&c->h_Lc, sizeof(Real) * 3 * K * S, hipHostMallocDefault);
    if (e != hipSuccess) return e;
    std::memset(c->h_C, 0, sizeof(Real) * 3 * K * S);
    std::memset(c->h_U, 0, sizeof(Real) * 2 * K * S);
    std::memset(c->h_Lc, 0, sizeof(Real) * 3 * K * S);
    c->h_vtx.resize(c->nv);
    for (int64_t i = 0; i < c->nv; ++i) c->h_vtx[i] = make_double4(c->vx[i], c->vy[i], c->hb[i], 0.0);
    return hipSuccess;
}

template <typename Real>
hipError_t enqueue_separated_hetero(Lanes &L, int mode, int in, int out, double tstage, double dt)
{
    swe_ctx *c = L.c;
    const int b = c->cfg.p_base, pm = c->cfg.p_max;
    const size_t w = sizeof(Real), S = c->stride, K = c->K;
    hipError_t e = host_mirrors<Real>(c);
    if (e != hipSuccess) return e;
    StageArgs<Real> a = make_args<Real>(c);
    a.mixed = 0;
    a.Cin = static_cast<const Real *>(c->d_C[in]);
    a.Uin = static_cast<const Real *>(c->d_U[in]);
    a.Cn = static_cast<const Real *>(c->d_C[0]);
    a.Cout = static_cast<Real *>(c->d_C[out]);
    a.Uout = static_cast<Real *>(c->d_U[out]);
    L.time(a, mode == MODE_STAGE2 ? 1 : 0, tstage, dt);
    a.inlist = c->d_inlist;
    a.Lb = static_cast<Real *>(c->d_Lb);
    a.Lc = static_cast<Real *>(c->d_Lc);
    // the correction stream waits for the previous stage, then brings the
    // input state of the neighbour and listed ranges down
    e = L.fork();
    const int64_t h0 = c->halo_start, l0 = c->n_unlisted, ne = c->ne;
    if (e == hipSuccess && ne > h0)
        e = hipMemcpy2DAsync(static_cast<char *>(c->h_C) + w * h0, w * S, static_cast<const char *>(c->d_C[in]) + w * h0,
                             w * S, w * (ne - h0), 3 * K, hipMemcpyDeviceToHost, c->s_corr);
    if (e == hipSuccess && ne > h0)
        e = hipMemcpy2DAsync(static_cast<char *>(c->h_U) + w * h0, w * S, static_cast<const char *>(c->d_U[in]) + w * h0,
                             w * S, w * (ne - h0), 2 * K, hipMemcpyDeviceToHost, c->s_corr);
    // the base pass over every element on the GPU meanwhile
    if (e == hipSuccess) e = launch_base<Real>(L, mode, a, c->ne);
    if (e == hipSuccess) e = hipStreamSynchronize(c->s_corr);
    if (e != hipSuccess) return e;
    // the correction of the listed elements on the host's threads
    StageArgs<Real> h = a;
    h.m.vtx = c->h_vtx.data();
    h.m.ev = c->ev.data();
    h.m.enb = c->nb_host.data();
    h.m.enbk = c->nbk_host.data();
    h.m.ep = nullptr;
    h.Cin = static_cast<const Real *>(c->h_C);
    h.Uin = static_cast<const Real *>(c->h_U);
    h.Lc = static_cast<Real *>(c->h_Lc);
    h.src = nullptr;
    int nt = c->cfg.host_threads;
    if (nt <= 0) {
        // every core this process may run on
        cpu_set_t set;
        CPU_ZERO(&set);
        nt = sched_getaffinity(0, sizeof(set), &set) == 0 ? CPU_COUNT(&set) : 1;
        nt = std::max(1, nt);
    }
    if (host_corr(b, pm, c->fp32, &h, dt, c->p.data(), (int)l0, (int)ne, nt) != 0) return hipErrorInvalidValue;
    // back up, then the epilogue joins base part and correction
    if (ne > l0)
        e = hipMemcpy2DAsync(static_cast<char *>(c->d_Lc) + w * l0, w * S, static_cast<const char *>(c->h_Lc) + w * l0,
                             w * S, w * (ne - l0), 3 * K, hipMemcpyHostToDevice, c->s_corr);
    if (e == hipSuccess) e = L.join();
    if (e != hipSuccess) return e;
    a.list = c->d_list;
    a.count = c->d_cnt;
    return launch_epi_all(b, pm, c->fp32, mode, &a, list_blocks(c), (int)c->ne, L.a);
}

// Order-partitioned stage: the base kernel does every element of order
// p_base whose neighbours are all of order p_base (branch A); each order's
// listed elements get their full stage from a kernel of that order, all on
// parallel branches; nothing needs joining afterwards but the next stage.
template <typename Real>
hipError_t enqueue_partitioned(Lanes &L, int mode, int in, int out, double tstage, double dt)
{
    swe_ctx *c = L.c;
    const int b = c->cfg.p_base, pm = c->cfg.p_max;
    StageArgs<Real> a = make_args<Real>(c);
    a.mixed = 0;
    a.Cin = static_cast<const Real *>(c->d_C[in]);
    a.Uin = static_cast<const Real *>(c->d_U[in]);
    a.Cn = static_cast<const Real *>(c->d_C[0]);
    a.Cout = static_cast<Real *>(c->d_C[out]);
    a.Uout = static_cast<Real *>(c->d_U[out]);
    L.time(a, mode == MODE_STAGE2 ? 1 : 0, tstage, dt);
    a.inlist = c->d_inlist;
    a.skip_listed = 1;
    hipError_t e = L.fork();
    if (e != hipSuccess) return e;
    // with the elements grouped (static order map) the unlisted ones are the
    // first n_unlisted: the base pass covers them only
    e = launch_base<Real>(L, mode, a, c->grouped ? c->n_unlisted : c->ne);
    if (e != hipSuccess) return e;
    // the listed elements of every order in one launch on branch B
    a.skip_listed = 0;
    a.list = c->d_list;
    a.count = c->d_cnt;
    e = launch_full_all(b, pm, c->fp32, mode, &a, list_blocks(c), (int)c->ne, L.side());
    if (e != hipSuccess) return e;
    return L.join();
}

// Minimum depth control over the stage output in buffer out (base branch,
// after everything the stage joined on it).
template <typename Real>
hipError_t enqueue_depth_limit(Lanes &L, int out)
{
    swe_ctx *c = L.c;
    StageArgs<Real> a = make_args<Real>(c);
    a.Cout = static_cast<Real *>(c->d_C[out]);
    a.Uout = static_cast<Real *>(c->d_U[out]);
    if (L.graph) a.inst = c->d_inst;
    return launch_depth_limit(c->cfg.p_max, c->fp32, &a, c->cfg.h_min, L.a);
}

// One SSP-RK2 step (order update first when adaptive).
template <typename Real>
hipError_t enqueue_step(Lanes &L, double tn, double dt)
{
    swe_ctx *c = L.c;
    hipError_t e = hipSuccess;
    if (c->cfg.adapt) {
        e = enqueue_adapt<Real>(L, tn);
        if (e != hipSuccess) return e;
    }
    for (int st = 0; st < 2 && e == hipSuccess; ++st) {
        const int mode = st == 0 ? MODE_STAGE1 : MODE_STAGE2, in = st, out = 1 - st;
        const double ts = tn + st * dt;
        if (separated(c) && c->cfg.separate == 2) e = enqueue_partitioned<Real>(L, mode, in, out, ts, dt);
        else if (separated(c) && c->cfg.hetero) e = enqueue_separated_hetero<Real>(L, mode, in, out, ts, dt);
        else if (separated(c)) e = enqueue_separated<Real>(L, mode, in, out, ts, dt);
        else e = enqueue_stage<Real>(L, mode, in, out, ts, dt, st ? c->d_C[0] : nullptr, nullptr);
        if (e == hipSuccess && c->cfg.h_min > 0.0) e = enqueue_depth_limit<Real>(L, out);
    }
    return e;
}

// The step graph: the device clock (stage times, open-sea elevation, depth
// check stop; an adaptive step's order update advances it), then one step as
// above.  Rebuilt when what it launches changes.
std::vector<long long> step_graph_key(const swe_ctx *c)
{
    return {(long long)(intptr_t)c->d_C[0], (long long)(intptr_t)c->d_src, c->uniform ? 1 : 0,
            c->list_cnt[0], c->list_cnt[1], c->list_cnt[2], c->list_cnt[3]};
}

// Steps per replay of the multi-step graph: the gap between two graph
// launches is several times that between two dependent nodes.
constexpr int GRAPH_STEPS = 8;

hipError_t build_graph(swe_ctx *c, int nsteps, hipGraph_t *g_out, hipGraphExec_t *x_out)
{
    hipGraph_t g = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e != hipSuccess) return e;
    Lanes L(c, g);
    for (int s = 0; s < nsteps && e == hipSuccess; ++s) {
        // an adaptive step's order update advances the clock itself
        if (!c->cfg.adapt) e = launch_batch_clock(c->d_inst, c->d_flag, 1, L.a);
        if (e == hipSuccess) e = c->fp32 ? enqueue_step<float>(L, 0.0, 0.0) : enqueue_step<double>(L, 0.0, 0.0);
    }
    if (e == hipSuccess) e = hipGraphInstantiate(x_out, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        *x_out = nullptr;
        return e;
    }
    *g_out = g;
    return hipSuccess;
}

swe_status ensure_step_graph(swe_ctx *c)
{
    const std::vector<long long> key = step_graph_key(c);
    if (c->step_exec && c->multi_exec && key == c->graph_key) return SWE_OK;
    drop_step_graph(c);
    hipError_t e = build_graph(c, 1, &c->step_graph, &c->step_exec);
    if (e == hipSuccess) e = build_graph(c, GRAPH_STEPS, &c->multi_graph, &c->multi_exec);
    if (e != hipSuccess) {
        drop_step_graph(c);
        return fail(c, SWE_EDEVICE, std::string("step graph: ") + hipGetErrorString(e));
    }
    c->graph_key = key;
    return SWE_OK;
}

// Elements whose right-hand side has a correction: order above p_base, or a
// neighbour above p_base.  Lists are grouped by order, ascending element index.
swe_status build_lists(swe_ctx *c)
{
    if (!separated(c)) return SWE_OK;
    const int b = c->cfg.p_base, S = c->stride;
    std::vector<unsigned char> in(S, 0);
    std::vector<std::vector<int>> L(4);
    for (int64_t i = 0; i < c->ne; ++i) {
        bool listed = c->p[i] > b;
        for (int k = 0; k < 3 && !listed; ++k) {
            const int nb = c->nb_host[(size_t)k * S + i];
            if (nb >= 0 && c->p[nb] > b) listed = true;
        }
        if (listed) {
            in[i] = 1;
            L[c->p[i]].push_back((int)i);
        }
    }
    for (int p = 0; p < 4; ++p) c->list_cnt[p] = (int)L[p].size();
    HIP_TRY(c, h2d(c, c->d_inlist, in.data(), S));
    for (int p = 0; p < 4; ++p) {
        c->list_off[p] = p * (int)c->ne;
        if (!L[p].empty())
            HIP_TRY(c, h2d(c, c->d_list + c->list_off[p], L[p].data(), sizeof(int) * L[p].size()));
    }
    HIP_TRY(c, h2d(c, c->d_cnt, c->list_cnt, sizeof(int) * 4));
    return SWE_OK;
}

template <typename Real>
hipError_t enqueue_usolve(swe_ctx *c, int buf)
{
    StageArgs<Real> a = make_args<Real>(c);
    a.Cin = static_cast<const Real *>(c->d_C[buf]);
    a.Uout = static_cast<Real *>(c->d_U[buf]);
    return launch_usolve(c->cfg.p_max, c->fp32, &a, c->s_base);
}

hipError_t usolve_buf(swe_ctx *c, int buf)
{
    return c->fp32 ? enqueue_usolve<float>(c, buf) : enqueue_usolve<double>(c, buf);
}

// The host copy of the element orders.  An adaptive context changes its
// orders on the device every step; whatever truncates or projects a state
// to each element's order reads them back first.
swe_status refresh_orders(swe_ctx *c)
{
    if (!c->cfg.adapt || !c->d_p) return SWE_OK;
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    HIP_TRY(c, d2h(c, c->p.data(), c->d_p, c->ne));
    return SWE_OK;
}

// host [elem][3][K] physical -> device SoA reference-scaled (buffer buf);
// modes above each element's current order are dropped
swe_status upload_state(swe_ctx *c, const double *coef, void *dst)
{
    if (swe_status st = refresh_orders(c)) return st;
    const int K = c->K, S = c->stride;
    const size_t n = (size_t)3 * K * S;
    std::vector<double> h(n, 0.0);
    for (int64_t ie = 0; ie < c->ne; ++ie) {
        const int ue = c->e_perm[ie];
        const int Ke = K_OF[c->p[ie]];
        const double inv = 1.0 / c->sfac[ie];
        for (int j = 0; j < 3; ++j)
            for (int q = 0; q < K; ++q) {
                double v = q < Ke ? coef[((size_t)ue * 3 + j) * K + q] : 0.0;
                if (!std::isfinite(v)) return fail(c, SWE_EINVAL, "non-finite coefficient in state");
                h[((size_t)j * K + q) * S + ie] = v * inv;
            }
    }
    if (c->fp32) {
        std::vector<float> f(n);
        for (size_t i = 0; i < n; ++i) f[i] = (float)h[i];
        HIP_TRY(c, h2d(c, dst, f.data(), n * sizeof(float)));
    } else {
        HIP_TRY(c, h2d(c, dst, h.data(), n * sizeof(double)));
    }
    return SWE_OK;
}

swe_status download(swe_ctx *c, const void *src, int ncomp, double *out, bool is_rhs)
{
    const int K = c->K, S = c->stride;
    const size_t n = (size_t)ncomp * K * S;
    std::vector<double> h(n);
    if (c->fp32) {
        std::vector<float> f(n);
        HIP_TRY(c, d2h(c, f.data(), src, n * sizeof(float)));
        for (size_t i = 0; i < n; ++i) h[i] = f[i];
    } else {
        HIP_TRY(c, d2h(c, h.data(), src, n * sizeof(double)));
    }
    (void)is_rhs;
    for (int64_t ie = 0; ie < c->ne; ++ie) {
        const int ue = c->e_perm[ie];
        for (int j = 0; j < ncomp; ++j)
            for (int q = 0; q < K; ++q)
                out[((size_t)ue * ncomp + j) * K + q] = h[((size_t)j * K + q) * S + ie] * c->sfac[ie];
    }
    return SWE_OK;
}

swe_status upload_vertices(swe_ctx *c)
{
    std::vector<double4> v(c->nv);
    for (int64_t i = 0; i < c->nv; ++i) v[i] = make_double4(c->vx[i], c->vy[i], c->hb[i], 0.0);
    HIP_TRY(c, h2d(c, c->d_vtx, v.data(), sizeof(double4) * c->nv));
    return SWE_OK;
}

swe_status upload_order(swe_ctx *c)
{
    std::vector<signed char> h(c->stride, (signed char)c->cfg.p_max);
    for (int64_t i = 0; i < c->ne; ++i) h[i] = c->p[i];
    c->uniform = true;
    for (int64_t i = 0; i < c->ne; ++i)
        if (c->p[i] != c->cfg.p_max) c->uniform = false;
    HIP_TRY(c, h2d(c, c->d_p, h.data(), c->stride));
    return SWE_OK;
}

template <typename Real>
hipError_t enqueue_rhs_split(swe_ctx *c, double t)
{
    const int b = c->cfg.p_base, pm = c->cfg.p_max;
    StageArgs<Real> a = make_args<Real>(c);
    a.mixed = 0;
    a.Cin = static_cast<const Real *>(c->d_C[1]);
    a.Uin = static_cast<const Real *>(c->d_U[1]);
    a.Lout = static_cast<Real *>(c->d_L);
    a.Lc = static_cast<Real *>(c->d_Lc);
    a.xihat = xi_hat(c, t);
    a.dt = 0.0;
    hipError_t e = launch_stage(b, c->fp32, MODE_RHS, false, &a, c->s_base);
    a.list = c->d_list;
    a.count = c->d_cnt;
    if (e == hipSuccess) {
        Sink k;
        k.s = c->s_base;
        e = launch_corr_all(b, pm, c->fp32, &a, 1.0, list_blocks(c), (int)c->ne, k);
    }
    return e;
}

#ifndef SWE_SHARED_FLUX
#define SWE_SHARED_FLUX 1
#endif
// Edge items of the shared-flux stage kernel for the current numbering
// (replacing any built before), for every block; or, when some block would
// hold more than the kernel takes, for the blocks of unlisted elements of a
// grouped numbering (the base pass of the partitioned scheme needs no more:
// listed elements of one order are seldom neighbours of each other, so their
// blocks hold many edges to outside); else none.
swe_status build_items(swe_ctx *c)
{
    if (c->d_items) (void)hipFree(c->d_items);
    if (c->d_item_off) (void)hipFree(c->d_item_off);
    c->d_items = nullptr;
    c->d_item_off = nullptr;
    c->item_blocks = 0;
    if (SWE_SHARED_FLUX && stage_sh_supported(c->cfg.p_max, c->fp32)) {
        const int64_t ne = c->ne;
        const int S = c->stride;
        // edge items per block of BLOCK elements, grouped by kind: pairs of
        // elements of the block (once, from the lower index), neighbours
        // outside the block, land edges, open edges.  Item j goes to lane
        // j % BLOCK, so each run of 64 items is one wave's: where the block
        // still fits in 2 BLOCK slots, every kind starts at a multiple of 64
        // (empty slots before it), and no wave computes two kinds' traces.
        const int64_t nblk = (ne + BLOCK - 1) / BLOCK;
        std::vector<unsigned> items;
        std::vector<int> ioff((size_t)nblk + 1, 0);
        items.reserve((size_t)ne * 2);
        std::vector<unsigned> group[4];
        for (int64_t bi = 0; bi < nblk; ++bi) {
            ioff[(size_t)bi] = (int)items.size();
            const int64_t e0 = bi * BLOCK, e1 = std::min<int64_t>(e0 + BLOCK, ne);
            for (auto &gk : group) gk.clear();
            for (int64_t ei = e0; ei < e1; ++ei)
                for (int k = 0; k < 3; ++k) {
                    const int n = c->nb_host[(size_t)k * S + ei];
                    unsigned kd;
                    int lb = 0, kb = 0;
                    if (n >= 0 && n / BLOCK == bi) {
                        if (n < ei) continue;      // the pair is taken from the lower index
                        kd = 0;
                        lb = (int)(n - e0);
                        kb = (c->nbk_host[ei] >> (2 * k)) & 3;
                    } else if (n >= 0) {
                        kd = 1;
                    } else if (n == NB_LAND) {
                        kd = 2;
                    } else {
                        kd = 3;
                    }
                    group[kd].push_back((unsigned)(ei - e0) | ((unsigned)k << 8) | ((unsigned)lb << 10) |
                                        ((unsigned)kb << 18) | (kd << 20));
                }
            // outside neighbours in the order of their index: consecutive
            // lanes then read nearby elements, which share cache lines
            // (1 % shorter FP64 stages at p = 2; FP32 unchanged)
            std::stable_sort(group[1].begin(), group[1].end(), [&](unsigned x, unsigned y) {
                const int nx = c->nb_host[(size_t)((x >> 8) & 3) * S + e0 + (x & 0xff)];
                const int ny = c->nb_host[(size_t)((y >> 8) & 3) * S + e0 + (y & 0xff)];
                return nx < ny;
            });
            size_t padded = 0;
            for (int kd = 0; kd < 4; ++kd)
                if (!group[kd].empty()) padded = (padded + 63) / 64 * 64 + group[kd].size();
            const bool align = padded <= (size_t)(2 * BLOCK);
            const size_t b0 = items.size();
            for (int kd = 0; kd < 4; ++kd) {
                if (group[kd].empty()) continue;
                while (align && (items.size() - b0) % 64 != 0) items.push_back(ITEM_PAD);
                items.insert(items.end(), group[kd].begin(), group[kd].end());
            }
        }
        ioff[(size_t)nblk] = (int)items.size();
        // the kernel takes at most two items per lane; a block with more
        // (a mesh ordering with long block boundaries) leaves the mesh to
        // the element-gather kernel
        // the leading blocks that fit; of a grouped numbering only those of
        // unlisted elements are worth keeping (the base pass takes the rest
        // of its range on the gather kernel), else all blocks or none
        int64_t cover = 0;
        while (cover < nblk && ioff[(size_t)cover + 1] - ioff[(size_t)cover] <= 2 * BLOCK) ++cover;
        if (cover < nblk) {
            cover = c->grouped ? std::min<int64_t>(cover, (c->n_unlisted + BLOCK - 1) / BLOCK) : 0;
            items.resize((size_t)ioff[(size_t)cover]);
            for (int64_t bi = cover + 1; bi <= nblk; ++bi) ioff[(size_t)bi] = (int)items.size();
        }
        if (cover > 0) {
            HIP_TRY(c, hipMalloc(&c->d_items, sizeof(unsigned) * std::max<size_t>(items.size(), 1)));
            HIP_TRY(c, hipMalloc(&c->d_item_off, sizeof(int) * ioff.size()));
            if (!items.empty()) HIP_TRY(c, h2d(c, c->d_items, items.data(), sizeof(unsigned) * items.size()));
            HIP_TRY(c, h2d(c, c->d_item_off, ioff.data(), sizeof(int) * ioff.size()));
            c->item_blocks = cover;
        }
    }
    return SWE_OK;
}

// The edge items cover the first nblocks blocks (0: every block).
bool items_cover(const swe_ctx *c, int64_t nblocks)
{
    const int64_t all = (c->ne + BLOCK - 1) / BLOCK;
    return c->d_items && c->item_blocks >= (nblocks > 0 ? std::min(nblocks, all) : all);
}

// Renumber the elements: new internal index i is the element at old index
// order[i].  Every element-indexed array kept here and on the device follows
// (the state itself is written again by the caller); step graphs are dropped.
swe_status relayout(swe_ctx *c, const std::vector<int> &order)
{
    const int64_t ne = c->ne;
    const int S = c->stride;
    std::vector<int> inew(ne);
    for (int64_t i = 0; i < ne; ++i) inew[order[i]] = (int)i;
    std::vector<double> src;
    if (c->d_src) {
        src.resize((size_t)ne * 3 * c->K);
        const swe_status st = download(c, c->d_src, 3, src.data(), false);
        if (st) return st;
    }
    std::vector<int> e_perm(ne), ev((size_t)3 * S, 0), nb((size_t)3 * S, NB_LAND);
    std::vector<unsigned char> nbk(S, 0);
    std::vector<double> sfac(ne);
    std::vector<signed char> pe(ne);
    for (int64_t i = 0; i < ne; ++i) {
        const int o = order[i];
        e_perm[i] = c->e_perm[o];
        sfac[i] = c->sfac[o];
        pe[i] = c->p[o];
        nbk[i] = c->nbk_host[o];
        for (int k = 0; k < 3; ++k) {
            ev[(size_t)k * S + i] = c->ev[(size_t)k * S + o];
            const int n = c->nb_host[(size_t)k * S + o];
            nb[(size_t)k * S + i] = n >= 0 ? inew[n] : n;
        }
    }
    c->e_perm.swap(e_perm);
    for (int64_t i = 0; i < ne; ++i) c->e_iperm[c->e_perm[i]] = (int)i;
    c->ev.swap(ev);
    c->nb_host.swap(nb);
    c->nbk_host.swap(nbk);
    c->sfac.swap(sfac);
    c->p.swap(pe);
    drop_step_graph(c);
    HIP_TRY(c, h2d(c, c->d_ev, c->ev.data(), sizeof(int) * 3 * S));
    HIP_TRY(c, h2d(c, c->d_nb, c->nb_host.data(), sizeof(int) * 3 * S));
    HIP_TRY(c, h2d(c, c->d_nbk, c->nbk_host.data(), S));
    swe_status st = build_items(c);
    if (st) return st;
    if (c->d_src) st = upload_state(c, src.data(), c->d_src);
    return st;
}

// Static order map of a separated context: unlisted elements first, then the
// listed elements of each order, every group in the current (Morton) order,
// so that each order's list is one contiguous range of element slots.
swe_status group_by_lists(swe_ctx *c)
{
    const int b = c->cfg.p_base, S = c->stride;
    const int64_t ne = c->ne;
    std::vector<unsigned char> listed(ne, 0);
    for (int64_t i = 0; i < ne; ++i) {
        bool l = c->p[i] > b;
        for (int k = 0; k < 3 && !l; ++k) {
            const int n = c->nb_host[(size_t)k * S + i];
            if (n >= 0 && c->p[n] > b) l = true;
        }
        listed[i] = l ? 1 : 0;
    }
    // groups: unlisted elements, then the listed elements of each order.
    // The unlisted neighbours of listed elements (which the list kernels
    // gather) form a group of their own just before the lists, in the lists'
    // order, so that consecutive lanes share cache lines; the base pass takes
    // that group on the gather kernel (a second launch).  Measured on the
    // 1/32 dam break p1-2 (order-partitioned): 290 -> 265 us per FP64 stage,
    // 183 -> 162 us FP32; the separated scheme has grouped them before.
    std::vector<std::vector<int>> grp(6);
    for (int64_t i = 0; i < ne; ++i) {
        if (listed[i]) {
            grp[2 + c->p[i]].push_back((int)i);
            continue;
        }
        bool halo = false;
        for (int k = 0; k < 3 && !halo; ++k) {
            const int n = c->nb_host[(size_t)k * S + i];
            if (n >= 0 && listed[n]) halo = true;
        }
        grp[halo ? 1 : 0].push_back((int)i);
    }
    std::vector<int> order;
    order.reserve(ne);
    for (const auto &g : grp) order.insert(order.end(), g.begin(), g.end());
    c->n_unlisted = (int64_t)(grp[0].size() + grp[1].size());
    c->halo_start = (int64_t)grp[0].size();
    c->grouped = true;
    for (int64_t i = 0; i < ne; ++i)
        if (order[i] != (int)i) return relayout(c, order);
    return SWE_OK;
}

// Device bytes of the arrays a context keeps as long as it has a mesh: vertex
// and neighbour ids, neighbour edges, orders, vertices, flag, clock, mass
// reduction scratch.
int64_t kept_bytes(int64_t ne, int64_t nv)
{
    const int64_t S = (ne + BLOCK - 1) / BLOCK * BLOCK;
    return 2 * 3 * 4 * S + 2 * S + 32 * nv + 4 + (int64_t)sizeof(InstDesc) + 8 * (S / BLOCK + 2);
}

// Device bytes of a context's state: C0, C1, U0, U1, the right-hand-side
// scratch and the shared-flux kernel's edge items (at most 3 per element).
int64_t state_bytes(int64_t ne, int p, bool fp32)
{
    const int64_t S = (ne + BLOCK - 1) / BLOCK * BLOCK;
    const int64_t K = K_OF[p], w = fp32 ? 4 : 8;
    int64_t b = (2 * 3 * K + 2 * 2 * K + 3 * K) * S * w;
    if (stage_sh_supported(p, fp32)) b += 3 * 4 * S + 4 * (S / BLOCK + 1);
    return b;
}

// Device bytes of a batch's pool of order p at capacity nc (elements):
// state and velocity ping-pong buffers, vertex and neighbour ids, neighbour
// edges, edge items and their block counts, tile list.
int64_t pool_bytes(int p, bool fp32, int64_t nc)
{
    if (nc <= 0) return 0;
    const int64_t K = K_OF[p], w = fp32 ? 4 : 8;
    int64_t b = (2 * 3 * K + 2 * 2 * K) * nc * w + 2 * 3 * 4 * nc + 3 * nc;
    if (stage_sh_supported(p, fp32)) b += 3 * 4 * nc + 4 * (nc / BLOCK);
    return b + (int64_t)sizeof(int2) * (nc / 64 + 1 + nc / BLOCK + 1);
}

}  // namespace

extern "C" {

void swe_config_default(swe_config *cfg)
{
    if (!cfg) return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->precision = SWE_FP64;
    cfg->p_base = 1;
    cfg->p_max = 1;
    cfg->g = 9.81;
    cfg->friction = SWE_FRICTION_NONE;
    cfg->adapt_tau = 1e-3;
    cfg->step_graph = 1;
}

swe_status swe_create(const swe_config *cfg, swe_ctx **out)
{
    if (!cfg || !out) return SWE_EINVAL;
    *out = nullptr;
    if (cfg->precision != SWE_FP64 && cfg->precision != SWE_FP32_WB) return SWE_EINVAL;
    if (cfg->p_max < 0 || cfg->p_max > 3 || cfg->p_base < 0 || cfg->p_base > cfg->p_max) return SWE_EINVAL;
    if (!(cfg->g > 0.0) || cfg->friction < 0 || cfg->friction > 2) return SWE_EINVAL;
    if (cfg->adapt && !(cfg->adapt_tau > 0.0)) return SWE_EINVAL;
    if (cfg->separate < 0 || cfg->separate > 2) return SWE_EINVAL;
    // heterogeneous stages: the order-separated scheme on a static order map
    if (cfg->hetero < 0 || cfg->hetero > 1 || cfg->host_threads < 0) return SWE_EINVAL;
    if (cfg->hetero && (cfg->separate != 1 || cfg->adapt || cfg->p_base >= cfg->p_max)) return SWE_EINVAL;
    if (!(cfg->h_min >= 0.0) || !std::isfinite(cfg->h_min)) return SWE_EINVAL;
    // FP32 order-partitioned stepping with orders up to 3 (its full-order
    // kernels k_full<p, 3, float>) is switched off: one run of it aborted on
    // the device and no cause has been found in the source.  The
    // order-separated scheme (separate = 1) covers the same runs.
    if (cfg->precision == SWE_FP32_WB && cfg->separate == 2 && cfg->p_max == 3 && cfg->p_base < 3)
        return SWE_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev <= 0) return SWE_EDEVICE;
    // the fixed array of swe_mass_noalloc: its address on this device, taken at set-up
    if (mass_scratch(nullptr) != hipSuccess) return SWE_EDEVICE;
    swe_ctx *c = new (std::nothrow) swe_ctx();
    if (!c) return SWE_ENOMEM;
    c->cfg = *cfg;
    c->fp32 = cfg->precision == SWE_FP32_WB;
    c->rsz = c->fp32 ? 4 : 8;
    c->K = K_OF[cfg->p_max];
    if (cfg->stream_base) {
        c->s_base = static_cast<hipStream_t>(cfg->stream_base);
    } else {
        if (hipStreamCreateWithFlags(&c->s_base, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return SWE_EDEVICE;
        }
        c->own_base = true;
    }
    if (cfg->stream_corr) {
        c->s_corr = static_cast<hipStream_t>(cfg->stream_corr);
    } else {
        if (hipStreamCreateWithFlags(&c->s_corr, hipStreamNonBlocking) != hipSuccess) {
            if (c->own_base) (void)hipStreamDestroy(c->s_base);
            delete c;
            return SWE_EDEVICE;
        }
        c->own_corr = true;
    }
    if (hipEventCreateWithFlags(&c->ev_ready, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->ev_corr, hipEventDisableTiming) != hipSuccess) {
        if (c->own_base) (void)hipStreamDestroy(c->s_base);
        if (c->own_corr) (void)hipStreamDestroy(c->s_corr);
        delete c;
        return SWE_EDEVICE;
    }
    *out = c;
    return SWE_OK;
}

void swe_destroy(swe_ctx *c)
{
    if (!c) return;
    if (c->s_base) (void)hipStreamSynchronize(c->s_base);
    if (c->s_corr) (void)hipStreamSynchronize(c->s_corr);
    free_mesh(c);
    if (c->ev_ready) (void)hipEventDestroy(c->ev_ready);
    if (c->ev_corr) (void)hipEventDestroy(c->ev_corr);
    if (c->own_base) (void)hipStreamDestroy(c->s_base);
    if (c->own_corr) (void)hipStreamDestroy(c->s_corr);
    delete c;
}

const char *swe_last_error(const swe_ctx *c) { return c ? c->err.c_str() : "null context"; }

int64_t swe_num_elements(const swe_ctx *c) { return c ? c->ne : 0; }
int swe_num_modes(const swe_ctx *c) { return c ? c->K : 0; }

int64_t swe_footprint_bytes(int64_t ne, int p_max, int precision)
{
    if (ne <= 0 || p_max < 0 || p_max > 3) return -1;
    const bool fp32 = precision == SWE_FP32_WB;
    const int64_t S = (ne + BLOCK - 1) / BLOCK * BLOCK;
    // vertices of a triangulated polygon: nv <= ne + 2; the margin covers a few holes
    const int64_t nv_est = ne + 2 * (int64_t)std::sqrt((double)ne) + 2;
    const int64_t kept = kept_bytes(ne, nv_est);
    // on its own: every array of the context; resident in an empty batch: its
    // share of the pool of its order, of the vertex pool, and what it keeps
    const int64_t alone = kept + state_bytes(ne, p_max, fp32);
    const int64_t resident = kept + pool_bytes(p_max, fp32, S) + 32 * nv_est;
    return std::max(alone, resident);
}

swe_status swe_set_mesh(swe_ctx *c, int64_t nv, const double *vxy, int64_t ne, const int32_t *tri,
                        const int8_t *tag)
{
    if (!c) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch");
    if (nv < 3 || ne < 1 || !vxy || !tri) return fail(c, SWE_EINVAL, "empty mesh");
    {
        // element arrays are addressed with 32-bit byte offsets (buffer resources)
        const int64_t S = (ne + BLOCK - 1) / BLOCK * BLOCK;
        if ((int64_t)3 * c->K * S * (int64_t)c->rsz > (int64_t)INT32_MAX)
            return fail(c, SWE_EUNSUPPORTED, "mesh too large: a coefficient array would exceed 2 GiB");
    }
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    HIP_TRY(c, hipStreamSynchronize(c->s_corr));
    free_mesh(c);
    for (int64_t e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k)
            if (tri[3 * e + k] < 0 || tri[3 * e + k] >= nv)
                return fail(c, SWE_EINVAL, "vertex id out of range in element " + std::to_string(e));
    // areas and Morton order of centroids
    std::vector<double> cx(ne), cy(ne);
    double xmin = 1e300, xmax = -1e300, ymin = 1e300, ymax = -1e300;
    for (int64_t e = 0; e < ne; ++e) {
        const int a = tri[3 * e], b = tri[3 * e + 1], d = tri[3 * e + 2];
        const double det = (vxy[2 * b] - vxy[2 * a]) * (vxy[2 * d + 1] - vxy[2 * a + 1]) -
                           (vxy[2 * d] - vxy[2 * a]) * (vxy[2 * b + 1] - vxy[2 * a + 1]);
        if (!(det > 0.0) || !std::isfinite(det))
            return fail(c, SWE_EINVAL, "element " + std::to_string(e) + " has non-positive area (must be counter-clockwise)");
        cx[e] = (vxy[2 * a] + vxy[2 * b] + vxy[2 * d]) / 3.0;
        cy[e] = (vxy[2 * a + 1] + vxy[2 * b + 1] + vxy[2 * d + 1]) / 3.0;
        xmin = std::min(xmin, cx[e]); xmax = std::max(xmax, cx[e]);
        ymin = std::min(ymin, cy[e]); ymax = std::max(ymax, cy[e]);
    }
    const double sx = xmax > xmin ? 65535.0 / (xmax - xmin) : 0.0;
    const double sy = ymax > ymin ? 65535.0 / (ymax - ymin) : 0.0;
    std::vector<uint64_t> key(ne);
    for (int64_t e = 0; e < ne; ++e) {
        const uint32_t ix = (uint32_t)((cx[e] - xmin) * sx), iy = (uint32_t)((cy[e] - ymin) * sy);
        key[e] = ((uint64_t)(spread16(ix) | (spread16(iy) << 1)) << 32) | (uint64_t)e;
    }
    std::sort(key.begin(), key.end());
    c->ne = ne;
    c->nv = nv;
    c->stride = (int)((ne + BLOCK - 1) / BLOCK * BLOCK);
    c->e_perm.assign(ne, 0);
    c->e_iperm.assign(ne, 0);
    for (int64_t i = 0; i < ne; ++i) {
        c->e_perm[i] = (int)(key[i] & 0xffffffffu);
        c->e_iperm[c->e_perm[i]] = (int)i;
    }
    // vertices in order of first use
    c->v_iperm.assign(nv, -1);
    c->v_perm.clear();
    c->v_perm.reserve(nv);
    for (int64_t i = 0; i < ne; ++i)
        for (int k = 0; k < 3; ++k) {
            const int v = tri[3 * (size_t)c->e_perm[i] + k];
            if (c->v_iperm[v] < 0) {
                c->v_iperm[v] = (int)c->v_perm.size();
                c->v_perm.push_back(v);
            }
        }
    for (int64_t v = 0; v < nv; ++v)
        if (c->v_iperm[v] < 0) {   // unused vertex: keep it at the end
            c->v_iperm[v] = (int)c->v_perm.size();
            c->v_perm.push_back((int)v);
        }
    c->vx.assign(nv, 0.0); c->vy.assign(nv, 0.0); c->hb.assign(nv, 0.0);
    for (int64_t i = 0; i < nv; ++i) {
        c->vx[i] = vxy[2 * (size_t)c->v_perm[i]];
        c->vy[i] = vxy[2 * (size_t)c->v_perm[i] + 1];
    }
    const int S = c->stride;
    c->ev.assign((size_t)3 * S, 0);
    c->sfac.assign(ne, 1.0);
    for (int64_t i = 0; i < ne; ++i) {
        const int ue = c->e_perm[i];
        for (int k = 0; k < 3; ++k) c->ev[(size_t)k * S + i] = c->v_iperm[tri[3 * (size_t)ue + k]];
        const int a = c->ev[i], b = c->ev[S + i], d = c->ev[2 * (size_t)S + i];
        const double det = (c->vx[b] - c->vx[a]) * (c->vy[d] - c->vy[a]) - (c->vx[d] - c->vx[a]) * (c->vy[b] - c->vy[a]);
        c->sfac[i] = std::sqrt(det);
    }
    // connectivity from shared vertex pairs
    std::vector<int> nb((size_t)3 * S, NB_LAND);
    std::vector<unsigned char> nbk(S, 0);
    std::unordered_map<uint64_t, int64_t> open;
    open.reserve((size_t)ne * 2);
    for (int64_t i = 0; i < ne; ++i)
        for (int k = 0; k < 3; ++k) {
            const int va = c->ev[(size_t)((k + 1) % 3) * S + i], vb = c->ev[(size_t)((k + 2) % 3) * S + i];
            const uint64_t lo = (uint64_t)std::min(va, vb), hi = (uint64_t)std::max(va, vb);
            const uint64_t key2 = (lo << 32) | hi;
            auto it = open.find(key2);
            if (it == open.end()) {
                open.emplace(key2, i * 3 + k);
            } else {
                const int64_t other = it->second;
                if (other < 0) return fail(c, SWE_EINVAL, "edge shared by more than two elements");
                const int64_t j = other / 3;
                const int kj = (int)(other % 3);
                nb[(size_t)k * S + i] = (int)j;
                nb[(size_t)kj * S + j] = (int)i;
                nbk[i] |= (unsigned char)(kj << (2 * k));
                nbk[j] |= (unsigned char)(k << (2 * kj));
                it->second = -1;
            }
        }
    for (int64_t i = 0; i < ne; ++i)
        for (int k = 0; k < 3; ++k)
            if (nb[(size_t)k * S + i] < 0) {
                const int ue = c->e_perm[i];
                const int tg = tag ? tag[3 * (size_t)ue + k] : -1;
                nb[(size_t)k * S + i] = tg == 1 ? NB_OPEN : NB_LAND;
            }
    // device buffers
    const size_t w = c->rsz, K = c->K;
    HIP_TRY(c, hipMalloc(&c->d_vtx, sizeof(double4) * nv));
    HIP_TRY(c, hipMalloc(&c->d_ev, sizeof(int) * 3 * S));
    HIP_TRY(c, hipMalloc(&c->d_nb, sizeof(int) * 3 * S));
    HIP_TRY(c, hipMalloc(&c->d_nbk, S));
    HIP_TRY(c, hipMalloc(&c->d_p, S));
    for (int b = 0; b < 2; ++b) {
        HIP_TRY(c, hipMalloc(&c->d_C[b], w * 3 * K * S));
        HIP_TRY(c, hipMalloc(&c->d_U[b], w * 2 * K * S));
        HIP_TRY(c, dzero(c, c->d_C[b], w * 3 * K * S));
        HIP_TRY(c, dzero(c, c->d_U[b], w * 2 * K * S));
    }
    HIP_TRY(c, hipMalloc(&c->d_L, w * 3 * K * S));
    HIP_TRY(c, hipMalloc(&c->d_flag, sizeof(int)));
    HIP_TRY(c, hipMalloc(&c->d_inst, sizeof(InstDesc)));
    HIP_TRY(c, dzero(c, c->d_flag, sizeof(int)));
    HIP_TRY(c, hipMalloc(&c->d_part, sizeof(double) * (mass_partials((int)ne) + 1)));
    HIP_TRY(c, hipMalloc(&c->d_mass, sizeof(double)));
    HIP_TRY(c, h2d(c, c->d_ev, c->ev.data(), sizeof(int) * 3 * S));
    HIP_TRY(c, h2d(c, c->d_nb, nb.data(), sizeof(int) * 3 * S));
    HIP_TRY(c, h2d(c, c->d_nbk, nbk.data(), S));
    c->nb_host = nb;
    c->nbk_host = nbk;
    c->grouped = false;
    c->n_unlisted = ne;
    swe_status st0 = SWE_OK;
    st0 = build_items(c);
    if (st0) return st0;
    if (separated(c) || c->cfg.adapt) {
        const int KB = K_OF[c->cfg.p_base];
        HIP_TRY(c, hipMalloc(&c->d_inlist, S));
        HIP_TRY(c, dzero(c, c->d_inlist, S));
        HIP_TRY(c, hipMalloc(&c->d_Lb, w * 3 * KB * S));
        HIP_TRY(c, hipMalloc(&c->d_Lc, w * 3 * K * S));
        HIP_TRY(c, hipMalloc(&c->d_list, sizeof(int) * 4 * (size_t)ne));
        HIP_TRY(c, hipMalloc(&c->d_cnt, sizeof(int) * 4));
        HIP_TRY(c, dzero(c, c->d_cnt, sizeof(int) * 4));
        HIP_TRY(c, hipMalloc(&c->d_pnew, S));
        HIP_TRY(c, hipMalloc(&c->d_I, sizeof(double) * S));
    }
    c->p.assign(ne, (signed char)(separated(c) ? c->cfg.p_base : c->cfg.p_max));
    swe_status st = upload_order(c);
    if (st) return st;
    st = build_lists(c);
    if (st) return st;
    st = upload_vertices(c);
    if (st) return st;
    c->t = 0.0;
    c->failed = false;
    c->have_mesh = true;
    return SWE_OK;
}

swe_status swe_set_bathymetry(swe_ctx *c, const double *hb)
{
    if (!c || !hb) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch");
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    for (int64_t i = 0; i < c->nv; ++i) {
        const double v = hb[c->v_perm[i]];
        if (!std::isfinite(v)) return fail(c, SWE_EINVAL, "non-finite bathymetry");
        c->hb[i] = v;
    }
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    swe_status st = upload_vertices(c);
    if (st) return st;
    // the velocity depends on the depth: recompute it for the current state
    HIP_TRY(c, usolve_buf(c, 0));
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    return SWE_OK;
}

swe_status swe_set_order(swe_ctx *c, const int8_t *p)
{
    if (!c || !p) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch");
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    for (int64_t e = 0; e < c->ne; ++e)
        if (p[e] < c->cfg.p_base || p[e] > c->cfg.p_max)
            return fail(c, SWE_EINVAL, "order out of [p_base, p_max] at element " + std::to_string(e));
    // keep the current state, truncated or extended to the new orders
    std::vector<double> coef((size_t)c->ne * 3 * c->K);
    double t = 0.0;
    swe_status st = swe_get_state(c, coef.data(), &t);
    if (st) return st;
    for (int64_t i = 0; i < c->ne; ++i) c->p[i] = p[c->e_perm[i]];
    if (separated(c) && !c->cfg.adapt) {
        st = group_by_lists(c);
        if (st) return st;
    }
    st = upload_order(c);
    if (st) return st;
    st = build_lists(c);
    if (st) return st;
    return swe_set_state(c, t, coef.data());
}

swe_status swe_get_order(swe_ctx *c, int8_t *p)
{
    if (!c || !p) return SWE_EINVAL;
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    if (swe_status st = refresh_orders(c)) return st;   // orders change on the device every step
    for (int64_t i = 0; i < c->ne; ++i) p[c->e_perm[i]] = c->p[i];
    return SWE_OK;
}

swe_status swe_set_open_boundary(swe_ctx *c, int ncon, const double *amp, const double *omega,
                                 const double *phase)
{
    if (!c || ncon < 0 || ncon > NCON_MAX) return SWE_EINVAL;
    if (ncon > 0 && (!amp || !omega || !phase)) return SWE_EINVAL;
    c->ncon = ncon;
    for (int i = 0; i < ncon; ++i) {
        c->amp[i] = amp[i];
        c->omega[i] = omega[i];
        c->phase[i] = phase[i];
    }
    return SWE_OK;
}

swe_status swe_set_state(swe_ctx *c, double t0, const double *coef)
{
    if (!c || !coef) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch");
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    HIP_TRY(c, hipStreamSynchronize(c->s_corr));
    swe_status st = upload_state(c, coef, c->d_C[0]);
    if (st) return st;
    // modes above each element's order are zero in every state buffer
    HIP_TRY(c, dzero(c, c->d_C[1], c->rsz * 3 * c->K * c->stride));
    HIP_TRY(c, dzero(c, c->d_U[1], c->rsz * 2 * c->K * c->stride));
    HIP_TRY(c, dzero(c, c->d_flag, sizeof(int)));
    HIP_TRY(c, usolve_buf(c, 0));
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    c->t = t0;
    c->failed = false;
    return SWE_OK;
}

swe_status swe_project_points(swe_ctx *c, double *xy)
{
    if (!c || !xy) return SWE_EINVAL;
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    const int S = c->stride;
    for (int64_t i = 0; i < c->ne; ++i) {
        const int ue = c->e_perm[i];
        const int a = c->ev[i], b = c->ev[S + i], d = c->ev[2 * (size_t)S + i];
        for (int q = 0; q < SWET_NQP; ++q) {
            xy[((size_t)ue * SWET_NQP + q) * 2] = c->vx[a] + QX[q] * (c->vx[b] - c->vx[a]) + QY[q] * (c->vx[d] - c->vx[a]);
            xy[((size_t)ue * SWET_NQP + q) * 2 + 1] = c->vy[a] + QX[q] * (c->vy[b] - c->vy[a]) + QY[q] * (c->vy[d] - c->vy[a]);
        }
    }
    return SWE_OK;
}

swe_status swe_set_state_points(swe_ctx *c, double t0, const double *vals)
{
    if (!c || !vals) return SWE_EINVAL;
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    if (swe_status st = refresh_orders(c)) return st;
    const int K = c->K;
    std::vector<double> coef((size_t)c->ne * 3 * K, 0.0);
    for (int64_t i = 0; i < c->ne; ++i) {
        const int ue = c->e_perm[i];
        const int Ke = K_OF[c->p[i]];
        const double s = c->sfac[i];
        for (int j = 0; j < 3; ++j)
            for (int m = 0; m < Ke; ++m) {
                double acc = 0.0;
                for (int q = 0; q < SWET_NQP; ++q)
                    acc += QW[q] * vals[((size_t)ue * SWET_NQP + q) * 3 + j] * QPHI[q][m];
                coef[((size_t)ue * 3 + j) * K + m] = acc * s;   // int f phi_e = s * int_ref f phi_ref
            }
    }
    return swe_set_state(c, t0, coef.data());
}

swe_status swe_set_source(swe_ctx *c, const double *coef)
{
    if (!c) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch");
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    if (!coef) {
        if (c->d_src) (void)hipFree(c->d_src);
        c->d_src = nullptr;
        return SWE_OK;
    }
    if (!c->d_src) HIP_TRY(c, hipMalloc(&c->d_src, c->rsz * 3 * c->K * c->stride));
    // a right-hand-side coefficient scales like the state
    return upload_state(c, coef, c->d_src);
}

swe_status swe_step(swe_ctx *c, int64_t nsteps, double dt)
{
    if (!c) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch");
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    if (c->failed) return fail(c, SWE_ESTATE, "context is in a failed state; call swe_set_state");
    if (nsteps < 0 || !(dt > 0.0) || !std::isfinite(dt)) return fail(c, SWE_EINVAL, "bad step count or dt");
    const double t0 = c->t;
    if (nsteps == 0) return SWE_OK;
    if (nsteps > INT_MAX) return fail(c, SWE_EINVAL, "too many steps in one call");
    if (c->cfg.adapt) c->uniform = false;   // orders may differ from the first order update on
    if (c->cfg.hetero && (!c->grouped || c->d_src))
        return fail(c, SWE_EINVAL, "heterogeneous stages need a static order map (swe_set_order) and no extra source");
    // graphs pay off where a step has many dependent kernels (order-separated
    // and order-partitioned steps); a fused step is two plain launches; a
    // heterogeneous stage waits for the host in the middle: launches
    const bool graph = c->ncon <= 4 && !c->cfg.hetero &&
                       (c->cfg.step_graph == 2 || (c->cfg.step_graph == 1 && separated(c)));
    if (graph) {
        swe_status st = ensure_step_graph(c);
        if (st != SWE_OK) return st;
        InstDesc d;
        std::memset(&d, 0, sizeof(d));
        d.ne = (int)c->ne;
        d.nv = (int)c->nv;
        d.order = c->cfg.p_max;
        d.active = 1;
        d.steps_left = (int)nsteps;
        d.ncon = c->ncon;
        for (int i = 0; i < c->ncon; ++i) {
            d.amp[i] = c->amp[i];
            d.omega[i] = c->omega[i];
            d.phase[i] = c->phase[i];
        }
        d.t0 = t0;
        d.t = t0;
        d.dt = dt;
        hipError_t e = launch_inst_set(c->d_inst, d, c->s_base);
        int64_t s = 0;
        for (; s + GRAPH_STEPS <= nsteps && e == hipSuccess; s += GRAPH_STEPS) e = hipGraphLaunch(c->multi_exec, c->s_base);
        for (; s < nsteps && e == hipSuccess; ++s) e = hipGraphLaunch(c->step_exec, c->s_base);
        if (e != hipSuccess) return fail(c, SWE_EDEVICE, std::string("step graph launch: ") + hipGetErrorString(e));
        c->t = t0 + (double)nsteps * dt;
        return SWE_OK;
    }
    Lanes L(c);
    for (int64_t s = 0; s < nsteps; ++s) {
        const double tn = t0 + (double)s * dt;
        const hipError_t e = c->fp32 ? enqueue_step<float>(L, tn, dt) : enqueue_step<double>(L, tn, dt);
        if (e != hipSuccess) return fail(c, SWE_EDEVICE, std::string("stage launch: ") + hipGetErrorString(e));
        c->t = t0 + (double)(s + 1) * dt;
    }
    return SWE_OK;
}

swe_status swe_sync(swe_ctx *c)
{
    if (!c) return SWE_EINVAL;
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    HIP_TRY(c, hipStreamSynchronize(c->s_corr));
    if (c->have_mesh) {
        int flag = 0;
        HIP_TRY(c, d2h(c, &flag, c->d_flag, sizeof(int)));
        if (flag) {
            c->failed = true;
            return fail(c, SWE_ESTATE, "non-finite value or non-positive mean depth detected");
        }
    }
    return SWE_OK;
}

swe_status swe_batch_sync(swe_batch *b);
double batch_member_time(swe_batch *b, int slot);

swe_status swe_get_state(swe_ctx *c, double *coef, double *t_out)
{
    if (!c || !coef) return SWE_EINVAL;
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    if (c->batch) {
        swe_status st = swe_batch_sync(c->batch);
        if (st != SWE_OK && st != SWE_ESTATE) return fail(c, st, "batch sync failed");
        c->t = batch_member_time(c->batch, c->slot);   // re-creates the state buffers for the copy
        if (!c->d_C[0]) return fail(c, SWE_EDEVICE, "state of the resident member could not be read");
    }
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    HIP_TRY(c, hipStreamSynchronize(c->s_corr));
    swe_status st = download(c, c->d_C[0], 3, coef, false);
    if (t_out) *t_out = c->t;
    if (c->batch) release_state_buffers(c);   // while resident the pool holds the state
    return st;
}

swe_status swe_mass(swe_ctx *c, double *out)
{
    if (!c || !out) return SWE_EINVAL;
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    if (c->batch) {
        swe_status st = swe_batch_sync(c->batch);
        if (st != SWE_OK && st != SWE_ESTATE) return fail(c, st, "batch sync failed");
        c->t = batch_member_time(c->batch, c->slot);   // also brings the state over from the pool
        if (!c->d_C[0]) return fail(c, SWE_EDEVICE, "state of the resident member could not be read");
    }
    HIP_TRY(c, launch_mass(view(c), c->fp32, c->d_C[0], c->d_part, c->d_mass, c->s_base));
    HIP_TRY(c, hipMemcpyAsync(out, c->d_mass, sizeof(double), hipMemcpyDeviceToHost, c->s_base));
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    if (c->batch) release_state_buffers(c);
    return SWE_OK;
}

swe_status swe_mass_noalloc(swe_ctx *c, double *d_out)
{
    if (!c || !d_out) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch (its state lives in the batch's pool)");
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    if (mass_partials((int)c->ne) > MASS_SCRATCH_PARTIALS)
        return fail(c, SWE_EINVAL, "swe_mass_noalloc takes at most " + std::to_string((int64_t)MASS_SCRATCH_PARTIALS * BLOCK) +
                                       " elements; this mesh has " + std::to_string(c->ne));
    HIP_TRY(c, launch_mass_noalloc(view(c), c->fp32, c->d_C[0], d_out, c->s_base));
    return SWE_OK;
}

swe_status swe_rhs(swe_ctx *c, double t, const double *coef, double *rhs)
{
    if (!c || !coef || !rhs) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch");
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    swe_status st = upload_state(c, coef, c->d_C[1]);
    if (st) return st;
    HIP_TRY(c, usolve_buf(c, 1));
    hipError_t e = c->fp32 ? enqueue_stage<float>(c, MODE_RHS, 1, -1, t, 0.0, nullptr, c->d_L)
                           : enqueue_stage<double>(c, MODE_RHS, 1, -1, t, 0.0, nullptr, c->d_L);
    if (e != hipSuccess) return fail(c, SWE_EDEVICE, std::string("rhs launch: ") + hipGetErrorString(e));
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    return download(c, c->d_L, 3, rhs, true);
}

swe_status swe_usolve(swe_ctx *c, const double *coef, double *u_out)
{
    if (!c || !coef || !u_out) return SWE_EINVAL;
    if (c->batch) return fail(c, SWE_EINVAL, "context is resident in a batch");
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    swe_status st = upload_state(c, coef, c->d_C[1]);
    if (st) return st;
    HIP_TRY(c, usolve_buf(c, 1));
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    return download(c, c->d_U[1], 2, u_out, false);
}

swe_status swe_rhs_split(swe_ctx *c, double t, const double *coef, double *base_out, double *corr_out)
{
    if (!c || !coef || !base_out || !corr_out) return SWE_EINVAL;
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    if (!separated(c)) return fail(c, SWE_EINVAL, "context is not order-separated (separate = 1, p_base < p_max)");
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    HIP_TRY(c, hipStreamSynchronize(c->s_corr));
    swe_status st = upload_state(c, coef, c->d_C[1]);
    if (st) return st;
    HIP_TRY(c, usolve_buf(c, 1));
    HIP_TRY(c, hipMemsetAsync(c->d_L, 0, c->rsz * 3 * c->K * c->stride, c->s_base));
    HIP_TRY(c, hipMemsetAsync(c->d_Lc, 0, c->rsz * 3 * c->K * c->stride, c->s_base));
    hipError_t e = c->fp32 ? enqueue_rhs_split<float>(c, t) : enqueue_rhs_split<double>(c, t);
    if (e != hipSuccess) return fail(c, SWE_EDEVICE, std::string("split rhs launch: ") + hipGetErrorString(e));
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    st = download(c, c->d_L, 3, base_out, true);
    if (st) return st;
    return download(c, c->d_Lc, 3, corr_out, true);
}

swe_status swe_indicator(swe_ctx *c, double t, const double *coef, double *I_out)
{
    if (!c || !coef || !I_out) return SWE_EINVAL;
    if (!c->have_mesh) return fail(c, SWE_EINVAL, "set_mesh first");
    if (!c->d_I) return fail(c, SWE_EINVAL, "indicator needs a context with adapt = 1");
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    HIP_TRY(c, hipStreamSynchronize(c->s_corr));
    swe_status st = upload_state(c, coef, c->d_C[1]);
    if (st) return st;
    hipError_t e;
    if (c->fp32) {
        StageArgs<float> a = make_args<float>(c);
        a.Cin = static_cast<const float *>(c->d_C[1]);
        a.xihat = xi_hat(c, t);
        e = launch_indicator(true, &a, 1.0, 0, 0, c->d_I, nullptr, c->s_base);
    } else {
        StageArgs<double> a = make_args<double>(c);
        a.Cin = static_cast<const double *>(c->d_C[1]);
        a.xihat = xi_hat(c, t);
        e = launch_indicator(false, &a, 1.0, 0, 0, c->d_I, nullptr, c->s_base);
    }
    if (e != hipSuccess) return fail(c, SWE_EDEVICE, std::string("indicator launch: ") + hipGetErrorString(e));
    std::vector<double> h(c->ne);
    HIP_TRY(c, hipStreamSynchronize(c->s_base));
    HIP_TRY(c, d2h(c, h.data(), c->d_I, sizeof(double) * c->ne));
    for (int64_t i = 0; i < c->ne; ++i) I_out[c->e_perm[i]] = h[i];
    return SWE_OK;
}


// ----------------------------------------------------------------------------
// Batches
// ----------------------------------------------------------------------------
}  // extern "C"

// A range allocator over [0, cap): first fit, coalescing frees.
struct RangeAlloc {
    std::vector<std::pair<int64_t, int64_t>> free;   // (start, length), sorted by start
    int64_t cap = 0;
    // where take(n) would place n elements, or -1 (nothing changes)
    int64_t find(int64_t n) const
    {
        for (const auto &r : free)
            if (r.second >= n) return r.first;
        return -1;
    }
    void clear()
    {
        free.clear();
        cap = 0;
    }
    int64_t take(int64_t n)
    {
        for (size_t k = 0; k < free.size(); ++k)
            if (free[k].second >= n) {
                const int64_t at = free[k].first;
                free[k].first += n;
                free[k].second -= n;
                if (free[k].second == 0) free.erase(free.begin() + k);
                return at;
            }
        return -1;
    }
    void give(int64_t at, int64_t n)
    {
        free.push_back({at, n});
        std::sort(free.begin(), free.end());
        std::vector<std::pair<int64_t, int64_t>> out;
        for (auto &r : free) {
            if (!out.empty() && out.back().first + out.back().second == r.first) out.back().second += r.second;
            else out.push_back(r);
        }
        free.swap(out);
    }
    void grow(int64_t newcap)
    {
        give(cap, newcap - cap);
        cap = newcap;
    }
};

struct swe_batch {
    swe_config cfg{};
    bool fp32 = false;
    size_t w = 8;
    int64_t budget = 0;
    // device bytes the batch holds: its pools (with growth slack), tile
    // lists, vertex pool and the arrays its members keep while resident;
    // never above budget, also while a pool grows (old and new arrays
    // coexist during the copy)
    int64_t alloc = 0;
    int cap = 0;
    hipStream_t s = nullptr;
    bool own_s = false;
    struct Member {
        swe_ctx *ctx = nullptr;
        bool mixed = false;            // per-element orders: a static order map or indicator-driven
        bool adapt = false;            // indicator-driven orders
        int64_t kept = 0;              // device bytes the member context keeps while resident
        int order = 0;
        int64_t first = 0, span = 0, vbase = 0, nv = 0;
        bool no_items = false;         // the context has no edge items (shared-flux kernel unusable)
    };
    std::vector<Member> mem;
    std::vector<InstDesc> h_inst;
    InstDesc *d_inst = nullptr;
    int *d_flags = nullptr;
    struct Pool { PoolView v{}; RangeAlloc ra; };
    Pool pool[4];
    double4 *d_vtx = nullptr;
    RangeAlloc vra;
    int2 *d_tiles[4] = {nullptr, nullptr, nullptr, nullptr};
    int tile_cap[4] = {0, 0, 0, 0};
    int *d_ntiles = nullptr;
    // 256-element tiles of the indicator-driven members of each order class
    int2 *d_atiles[4] = {nullptr, nullptr, nullptr, nullptr};
    int atile_cap[4] = {0, 0, 0, 0};
    int natiles[4] = {0, 0, 0, 0};
    int *d_natiles = nullptr;
    int mixed_members[4] = {0, 0, 0, 0};   // resident members of the order with per-element orders
    int tile[4] = {256, 256, 256, 256};
    bool shared[4] = {false, true, true, true};     // shared-flux kernel (256-element tiles) chosen for the order
    int no_items[4] = {0, 0, 0, 0};    // resident members of the order without edge items
    int grid[4] = {0, 0, 0, 0};
    int ntiles[4] = {0, 0, 0, 0};
    int ncu = 256;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int graph_orders = -1;             // bit p set: order p launched by the step graph
    std::string err;
};

namespace {

constexpr int POOL_ALIGN = 256;           // element ranges start on tile boundaries of every size

swe_status bfail(swe_batch *b, swe_status s, const std::string &msg)
{
    if (b) b->err = msg;
    return s;
}

#define BHIP_TRY(bb, expr)                                                                        \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess)                                                                     \
            return bfail((bb), e_ == hipErrorOutOfMemory ? SWE_ENOMEM : SWE_EDEVICE,              \
                         std::string(#expr) + ": " + hipGetErrorString(e_));                     \
    } while (0)

void drop_graph(swe_batch *b)
{
    if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
    if (b->graph) (void)hipGraphDestroy(b->graph);
    b->gexec = nullptr;
    b->graph = nullptr;
    b->graph_orders = -1;
}

// Capacity of a pool that has to hold need elements: twice the current one
// when the budget allows it, else need itself; 0 when even that does not
// fit.  room is what the pool's arrays may take (the old arrays stay
// allocated while they are copied, so the whole new size counts).
template <typename F>
int64_t grown_capacity(int64_t cap, int64_t need, int64_t room, F bytes)
{
    const int64_t twice = std::max(need, 2 * cap);
    if (bytes(twice) <= room) return twice;
    return bytes(need) <= room ? need : 0;
}

// Grow the pool of order p to capacity nc (a multiple of POOL_ALIGN).
swe_status grow_pool(swe_batch *b, int p, int64_t nc)
{
    swe_batch::Pool &P = b->pool[p];
    if (nc <= P.ra.cap) return SWE_OK;
    const int64_t K = K_OF[p];
    if ((int64_t)3 * K * nc * (int64_t)b->w > (int64_t)INT32_MAX)
        return bfail(b, SWE_EUNSUPPORTED, "pool of one order would exceed 2 GiB per array");
    PoolView v{};
    v.cap = (int)nc;
    BHIP_TRY(b, hipMalloc(&v.C0, b->w * 3 * K * nc));
    BHIP_TRY(b, hipMalloc(&v.C1, b->w * 3 * K * nc));
    BHIP_TRY(b, hipMalloc(&v.U0, b->w * 2 * K * nc));
    BHIP_TRY(b, hipMalloc(&v.U1, b->w * 2 * K * nc));
    BHIP_TRY(b, hipMalloc(&v.ev, sizeof(int) * 3 * nc));
    BHIP_TRY(b, hipMalloc(&v.nb, sizeof(int) * 3 * nc));
    BHIP_TRY(b, hipMalloc(&v.nbk, nc));
    BHIP_TRY(b, hipMalloc(&v.ep, nc));
    BHIP_TRY(b, hipMalloc(&v.pnew, nc));
    if (stage_sh_supported(p, b->fp32)) {
        BHIP_TRY(b, hipMalloc(&v.items, sizeof(unsigned) * 3 * nc));
        BHIP_TRY(b, hipMalloc(&v.nitems, sizeof(int) * (nc / BLOCK)));
        BHIP_TRY(b, hipMemsetAsync(v.nitems, 0, sizeof(int) * (nc / BLOCK), b->s));
    }
    BHIP_TRY(b, hipMemsetAsync(v.C1, 0, b->w * 3 * K * nc, b->s));
    BHIP_TRY(b, hipMemsetAsync(v.U1, 0, b->w * 2 * K * nc, b->s));
    const int64_t oc = P.ra.cap;
    if (oc > 0) {
        BHIP_TRY(b, hipMemcpy2DAsync(v.C0, b->w * nc, P.v.C0, b->w * oc, b->w * oc, 3 * K, hipMemcpyDeviceToDevice, b->s));
        BHIP_TRY(b, hipMemcpy2DAsync(v.U0, b->w * nc, P.v.U0, b->w * oc, b->w * oc, 2 * K, hipMemcpyDeviceToDevice, b->s));
        BHIP_TRY(b, hipMemcpy2DAsync(v.ev, 4 * nc, P.v.ev, 4 * oc, 4 * oc, 3, hipMemcpyDeviceToDevice, b->s));
        BHIP_TRY(b, hipMemcpy2DAsync(v.nb, 4 * nc, P.v.nb, 4 * oc, 4 * oc, 3, hipMemcpyDeviceToDevice, b->s));
        BHIP_TRY(b, hipMemcpyAsync(v.nbk, P.v.nbk, oc, hipMemcpyDeviceToDevice, b->s));
        BHIP_TRY(b, hipMemcpyAsync(v.ep, P.v.ep, oc, hipMemcpyDeviceToDevice, b->s));
        if (v.items) {
            BHIP_TRY(b, hipMemcpyAsync(v.items, P.v.items, sizeof(unsigned) * 3 * oc, hipMemcpyDeviceToDevice, b->s));
            BHIP_TRY(b, hipMemcpyAsync(v.nitems, P.v.nitems, sizeof(int) * (oc / BLOCK), hipMemcpyDeviceToDevice, b->s));
        }
        BHIP_TRY(b, hipStreamSynchronize(b->s));
        void *old[] = {P.v.C0, P.v.C1, P.v.U0, P.v.U1, P.v.ev, P.v.nb, P.v.nbk, P.v.ep, P.v.pnew, P.v.items,
                       P.v.nitems};
        for (void *q : old) (void)hipFree(q);
    }
    b->alloc += pool_bytes(p, b->fp32, nc) - pool_bytes(p, b->fp32, oc);
    P.v = v;
    P.ra.grow(nc);
    // tile list capacity follows the pool: at most one tile per 64 elements
    const int tc = (int)(nc / 64 + 1);
    int2 *nt = nullptr;
    BHIP_TRY(b, hipMalloc(&nt, sizeof(int2) * tc));
    if (b->d_tiles[p]) (void)hipFree(b->d_tiles[p]);
    b->d_tiles[p] = nt;
    b->tile_cap[p] = tc;
    const int ac = (int)(nc / BLOCK + 1);
    int2 *na = nullptr;
    BHIP_TRY(b, hipMalloc(&na, sizeof(int2) * ac));
    if (b->d_atiles[p]) (void)hipFree(b->d_atiles[p]);
    b->d_atiles[p] = na;
    b->atile_cap[p] = ac;
    drop_graph(b);
    return SWE_OK;
}

// Grow the vertex pool to capacity nc.
swe_status grow_vertices(swe_batch *b, int64_t nc)
{
    if (nc <= b->vra.cap) return SWE_OK;
    double4 *v = nullptr;
    BHIP_TRY(b, hipMalloc(&v, sizeof(double4) * nc));
    if (b->vra.cap) {
        BHIP_TRY(b, hipMemcpyAsync(v, b->d_vtx, sizeof(double4) * b->vra.cap, hipMemcpyDeviceToDevice, b->s));
        BHIP_TRY(b, hipStreamSynchronize(b->s));
        (void)hipFree(b->d_vtx);
    }
    b->alloc += (int64_t)sizeof(double4) * (nc - b->vra.cap);
    b->d_vtx = v;
    b->vra.grow(nc);
    drop_graph(b);
    return SWE_OK;
}

// Free the pool of order p (no member of that order is resident).
void release_pool(swe_batch *b, int p)
{
    swe_batch::Pool &P = b->pool[p];
    if (P.ra.cap == 0) return;
    void *q[] = {P.v.C0, P.v.C1, P.v.U0, P.v.U1, P.v.ev, P.v.nb, P.v.nbk, P.v.ep, P.v.pnew, P.v.items, P.v.nitems,
                 b->d_tiles[p], b->d_atiles[p]};
    for (void *x : q)
        if (x) (void)hipFree(x);
    b->alloc -= pool_bytes(p, b->fp32, P.ra.cap);
    P.v = PoolView{};
    P.ra.clear();
    b->d_tiles[p] = nullptr;
    b->tile_cap[p] = 0;
    b->d_atiles[p] = nullptr;
    b->atile_cap[p] = 0;
    drop_graph(b);
}

void release_vertices(swe_batch *b)
{
    if (b->vra.cap == 0) return;
    (void)hipFree(b->d_vtx);
    b->alloc -= (int64_t)sizeof(double4) * b->vra.cap;
    b->d_vtx = nullptr;
    b->vra.clear();
    drop_graph(b);
}

// Order p runs the shared-flux batch kernel: chosen for it, and every resident
// member of that order brought its edge items.
bool use_shared(const swe_batch *b, int p)
{
    // the shared-flux kernel takes uniform-order members only
    return b->shared[p] && b->no_items[p] == 0 && b->mixed_members[p] == 0 && b->pool[p].v.items != nullptr;
}

// Tile size of order p: 256 for the shared-flux kernel (tiles are its blocks).
int tile_of(const swe_batch *b, int p) { return use_shared(b, p) ? BLOCK : b->tile[p]; }

// Tile lists of the resident set: order p gets tiles of tile_of(b, p) elements.
swe_status upload_tiles(swe_batch *b)
{
    for (int p = 0; p < 4; ++p) {
        std::vector<int2> t;
        for (int i = 0; i < b->cap; ++i) {
            const swe_batch::Member &m = b->mem[i];
            if (!m.ctx || m.order != p) continue;
            for (int64_t f = 0; f < m.ctx->ne; f += tile_of(b, p)) t.push_back(make_int2(i, (int)(m.first + f)));
        }
        if ((int)t.size() > b->tile_cap[p]) return bfail(b, SWE_ENOMEM, "tile list capacity exceeded");
        b->ntiles[p] = (int)t.size();
        if (!t.empty())
            BHIP_TRY(b, hipMemcpyAsync(b->d_tiles[p], t.data(), sizeof(int2) * t.size(), hipMemcpyHostToDevice, b->s));
        if (b->grid[p] <= 0) b->grid[p] = 2 * b->ncu;
        // the order update's tiles: 256 elements of an indicator-driven member
        std::vector<int2> at;
        for (int i = 0; i < b->cap; ++i) {
            const swe_batch::Member &m = b->mem[i];
            if (!m.ctx || m.order != p || !m.adapt) continue;
            for (int64_t f = 0; f < m.ctx->ne; f += BLOCK) at.push_back(make_int2(i, (int)(m.first + f)));
        }
        if ((int)at.size() > b->atile_cap[p]) return bfail(b, SWE_ENOMEM, "tile list capacity exceeded");
        b->natiles[p] = (int)at.size();
        if (!at.empty())
            BHIP_TRY(b, hipMemcpyAsync(b->d_atiles[p], at.data(), sizeof(int2) * at.size(), hipMemcpyHostToDevice,
                                       b->s));
    }
    BHIP_TRY(b, hipMemcpyAsync(b->d_ntiles, b->ntiles, sizeof(int) * 4, hipMemcpyHostToDevice, b->s));
    BHIP_TRY(b, hipMemcpyAsync(b->d_natiles, b->natiles, sizeof(int) * 4, hipMemcpyHostToDevice, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    int present = 0;
    for (int p = 0; p < 4; ++p) present |= (b->ntiles[p] ? 1 << p : 0) | (b->natiles[p] ? 1 << (4 + p) : 0);
    if (present != b->graph_orders) drop_graph(b);   // the step graph launches other orders
    return SWE_OK;
}

// Grid of a batch stage launch: one block per tile the pool of order p can
// hold with tiles of `tile` elements, plus 8 (each XCD then has a block for
// every tile of its eighth of the list; surplus blocks exit at once).
int tile_grid(const swe_batch *b, int p, int tile)
{
    return (int)(b->pool[p].v.cap / tile) + 1 + 8;
}

BatchArgs batch_args(const swe_batch *b, int p)
{
    BatchArgs a;
    a.pool = b->pool[p].v;
    a.vtx = b->d_vtx;
    a.inst = b->d_inst;
    a.tiles = b->d_tiles[p];
    a.ntiles = b->d_ntiles + p;
    a.atiles = b->d_atiles[p];
    a.natiles = b->d_natiles + p;
    a.flags = b->d_flags;
    return a;
}

// Every order class runs in the multi-instance kernel (one tile per block).
// The single-instance path below (one launch per instance, clock and element
// offset read from the device) stays available for a class that cannot; a
// persistent kernel looping over tiles around the register-spilling order-3
// evaluation gave wrong results, the one-tile-per-block kernel does not loop.
bool per_instance(const swe_batch *b, int p)
{
    (void)b;
    (void)p;
    return false;
}

template <typename Real>
hipError_t instance_stage(swe_batch *b, int i, int mode, Sink &k)
{
    const swe_batch::Member &m = b->mem[i];
    const PoolView &v = b->pool[m.order].v;
    StageArgs<Real> a;
    std::memset(&a, 0, sizeof(a));
    a.m.ne = (int)m.ctx->ne;
    a.m.stride = v.cap;
    a.m.KS = K_OF[m.order];
    a.m.vtx = b->d_vtx;
    a.m.ev = v.ev;
    a.m.enb = v.nb;
    a.m.enbk = v.nbk;
    a.Cin = static_cast<const Real *>(mode == MODE_STAGE1 ? v.C0 : v.C1);
    a.Uin = static_cast<const Real *>(mode == MODE_STAGE1 ? v.U0 : v.U1);
    a.Cn = static_cast<const Real *>(v.C0);
    a.Cout = static_cast<Real *>(mode == MODE_STAGE1 ? v.C1 : v.C0);
    a.Uout = static_cast<Real *>(mode == MODE_STAGE1 ? v.U1 : v.U0);
    a.ph = b->h_inst[i].ph;
    a.flag = b->d_flags + i;
    a.inst = b->d_inst + i;
    a.e_off = (int)m.first;
    return launch_stage(m.order, b->fp32, mode, false, &a, k);
}

hipError_t enqueue_instance_stage(swe_batch *b, int i, int mode, Sink &k)
{
    return b->fp32 ? instance_stage<float>(b, i, mode, k) : instance_stage<double>(b, i, mode, k);
}

hipError_t enqueue_batch_step(swe_batch *b, Sink &k)
{
    hipError_t e = launch_batch_clock(b->d_inst, b->d_flags, b->cap, k);
    // order update of the indicator-driven members: every indicator before
    // any order is applied (an element's list flag reads its neighbours' new orders)
    for (int p = 1; p < 4 && e == hipSuccess; ++p)
        if (b->natiles[p]) e = launch_batch_indicator(b->fp32, batch_args(b, p), tile_grid(b, p, BLOCK), k);
    for (int p = 1; p < 4 && e == hipSuccess; ++p)
        if (b->natiles[p]) e = launch_batch_apply(p, b->fp32, batch_args(b, p), tile_grid(b, p, BLOCK), k);
    for (int mode = MODE_STAGE1; mode <= MODE_STAGE2 && e == hipSuccess; ++mode)
        for (int p = 0; p < 4 && e == hipSuccess; ++p) {
            if (b->ntiles[p] == 0) continue;
            if (per_instance(b, p)) {
                for (int i = 0; i < b->cap && e == hipSuccess; ++i)
                    if (b->mem[i].ctx && b->mem[i].order == p) e = enqueue_instance_stage(b, i, mode, k);
                continue;
            }
            // the kernels read the tile counts from device memory, so the grid
            // need not match the current resident set
            if (use_shared(b, p))
                e = launch_batch_stage_sh(p, b->fp32, mode, batch_args(b, p), tile_grid(b, p, BLOCK), k);
            else
                e = launch_batch_stage(p, b->fp32, mode, b->tile[p], batch_args(b, p), tile_grid(b, p, b->tile[p]), k);
        }
    return e;
}

// Build one step as a graph of kernel nodes in launch order (no stream
// capture); the kernels read everything that changes (times, budgets, tile
// counts) from device memory.
swe_status build_step_graph(swe_batch *b)
{
    drop_graph(b);
    hipGraph_t g = nullptr;
    BHIP_TRY(b, hipGraphCreate(&g, 0));
    Sink k;
    k.g = g;
    const hipError_t e = enqueue_batch_step(b, k);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return bfail(b, SWE_EDEVICE, std::string("step graph: ") + hipGetErrorString(e));
    }
    b->graph = g;
    BHIP_TRY(b, hipGraphInstantiate(&b->gexec, g, nullptr, nullptr, 0));
    b->graph_orders = 0;
    for (int p = 0; p < 4; ++p) b->graph_orders |= (b->ntiles[p] ? 1 << p : 0) | (b->natiles[p] ? 1 << (4 + p) : 0);
    return SWE_OK;
}

swe_status put_desc(swe_batch *b, int i)
{
    BHIP_TRY(b, hipMemcpyAsync(b->d_inst + i, &b->h_inst[i], sizeof(InstDesc), hipMemcpyHostToDevice, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    return SWE_OK;
}

swe_status get_desc(swe_batch *b, int i)
{
    BHIP_TRY(b, hipMemcpyAsync(&b->h_inst[i], b->d_inst + i, sizeof(InstDesc), hipMemcpyDeviceToHost, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    return SWE_OK;
}

// copy a resident instance's state and velocity from the pool into its
// context (whose state buffers are re-created for it)
swe_status pull_state(swe_batch *b, int i)
{
    const swe_batch::Member &m = b->mem[i];
    swe_ctx *c = m.ctx;
    const swe_batch::Pool &P = b->pool[m.order];
    const size_t w = b->w, K = c->K;
    if (swe_status st = restore_state_buffers(c)) return bfail(b, st, c->err);
    BHIP_TRY(b, hipMemcpy2DAsync(c->d_C[0], w * c->stride, static_cast<char *>(P.v.C0) + w * m.first, w * P.v.cap,
                                 w * c->ne, 3 * K, hipMemcpyDeviceToDevice, b->s));
    BHIP_TRY(b, hipMemcpy2DAsync(c->d_U[0], w * c->stride, static_cast<char *>(P.v.U0) + w * m.first, w * P.v.cap,
                                 w * c->ne, 2 * K, hipMemcpyDeviceToDevice, b->s));
    if (m.adapt)   // the orders the indicator chose while resident
        BHIP_TRY(b, hipMemcpyAsync(c->d_p, P.v.ep + m.first, c->ne, hipMemcpyDeviceToDevice, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    return SWE_OK;
}

}  // namespace

double batch_member_time(swe_batch *b, int slot)
{
    if (!b || slot < 0 || slot >= b->cap) return 0.0;
    if (get_desc(b, slot) != SWE_OK) return 0.0;
    if (pull_state(b, slot) != SWE_OK) return b->h_inst[slot].t;
    return b->h_inst[slot].t;
}

extern "C" {

swe_status swe_batch_create(const swe_config *cfg, int64_t budget, int max_instances, swe_batch **out)
{
    if (!cfg || !out || budget <= 0 || max_instances <= 0 || max_instances > 65536) return SWE_EINVAL;
    if (cfg->precision != SWE_FP64 && cfg->precision != SWE_FP32_WB) return SWE_EINVAL;
    *out = nullptr;
    swe_batch *b = new (std::nothrow) swe_batch();
    if (!b) return SWE_ENOMEM;
    b->cfg = *cfg;
    b->fp32 = cfg->precision == SWE_FP32_WB;
    b->w = b->fp32 ? 4 : 8;
    b->budget = budget;
    b->cap = max_instances;
    b->mem.assign(max_instances, swe_batch::Member());
    b->h_inst.assign(max_instances, InstDesc());
    std::memset(b->h_inst.data(), 0, sizeof(InstDesc) * max_instances);
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        b->ncu = prop.multiProcessorCount;
    if (cfg->stream_base) {
        b->s = static_cast<hipStream_t>(cfg->stream_base);
    } else if (hipStreamCreateWithFlags(&b->s, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return SWE_EDEVICE;
    } else {
        b->own_s = true;
    }
    if (hipMalloc(&b->d_inst, sizeof(InstDesc) * max_instances) != hipSuccess ||
        hipMalloc(&b->d_flags, sizeof(int) * max_instances) != hipSuccess ||
        hipMalloc(&b->d_ntiles, sizeof(int) * 4) != hipSuccess ||
        hipMalloc(&b->d_natiles, sizeof(int) * 4) != hipSuccess) {
        swe_batch_destroy(b);
        return SWE_ENOMEM;
    }
    if (hipMemcpyAsync(b->d_inst, b->h_inst.data(), sizeof(InstDesc) * max_instances, hipMemcpyHostToDevice,
                       b->s) != hipSuccess ||
        hipMemsetAsync(b->d_flags, 0, sizeof(int) * max_instances, b->s) != hipSuccess ||
        hipMemsetAsync(b->d_ntiles, 0, sizeof(int) * 4, b->s) != hipSuccess ||
        hipMemsetAsync(b->d_natiles, 0, sizeof(int) * 4, b->s) != hipSuccess ||
        hipStreamSynchronize(b->s) != hipSuccess) {
        swe_batch_destroy(b);
        return SWE_EDEVICE;
    }
    *out = b;
    return SWE_OK;
}

void swe_batch_destroy(swe_batch *b)
{
    if (!b) return;
    if (b->s) (void)hipStreamSynchronize(b->s);
    for (int i = 0; i < b->cap; ++i)
        if (b->mem[i].ctx) {
            swe_ctx *c = b->mem[i].ctx;
            (void)pull_state(b, i);
            (void)get_desc(b, i);
            c->t = b->h_inst[i].t;
            c->batch = nullptr;
            c->slot = -1;
            (void)build_items(c);
        }
    drop_graph(b);
    std::vector<void *> ptrs = {b->d_inst, b->d_flags, b->d_ntiles, b->d_natiles, b->d_vtx};
    for (int p = 0; p < 4; ++p) {
        const PoolView &v = b->pool[p].v;
        for (void *q : {v.C0, v.C1, v.U0, v.U1, (void *)v.ev, (void *)v.nb, (void *)v.nbk, (void *)v.ep,
                        (void *)v.pnew, (void *)v.items, (void *)v.nitems, (void *)b->d_tiles[p],
                        (void *)b->d_atiles[p]})
            ptrs.push_back(q);
    }
    for (void *q : ptrs)
        if (q) (void)hipFree(q);
    if (b->own_s) (void)hipStreamDestroy(b->s);
    delete b;
}

const char *swe_batch_last_error(const swe_batch *b) { return b ? b->err.c_str() : "null batch"; }
int64_t swe_batch_free_bytes(const swe_batch *b) { return b ? b->budget - b->alloc : 0; }

int swe_batch_resident(const swe_batch *b)
{
    if (!b) return 0;
    int n = 0;
    for (const auto &m : b->mem) n += m.ctx ? 1 : 0;
    return n;
}

swe_status swe_batch_admit(swe_batch *b, swe_ctx *c, int64_t nsteps, double dt, int32_t *slot)
{
    if (!b || !c || !slot || nsteps < 0 || !(dt > 0.0)) return SWE_EINVAL;
    if (!c->have_mesh) return bfail(b, SWE_EINVAL, "context has no mesh");
    if (c->batch) return bfail(b, SWE_EINVAL, "context is already resident in a batch");
    if (c->fp32 != b->fp32) return bfail(b, SWE_EINVAL, "context precision differs from the batch");
    if (c->cfg.separate || c->d_src || c->failed)
        return bfail(b, SWE_EINVAL, "batch members run the fused scheme (separate = 0) and take no extra source");
    if (c->ncon > 4) return bfail(b, SWE_EINVAL, "batch members support at most 4 forcing constituents");
    if (c->cfg.h_min > 0.0) return bfail(b, SWE_EINVAL, "batch members take no minimum depth control (h_min = 0)");
    int i = 0;
    while (i < b->cap && b->mem[i].ctx) ++i;
    if (i == b->cap) return bfail(b, SWE_ENOMEM, "no free slot");
    BHIP_TRY(b, hipStreamSynchronize(c->s_base));
    BHIP_TRY(b, hipStreamSynchronize(c->s_corr));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    // what admission takes from the budget, decided before anything changes:
    // the arrays the member keeps, growth of its order's pool and of the
    // vertex pool (each counted whole while its old arrays are copied)
    const int p = c->cfg.p_max;
    swe_batch::Pool &P = b->pool[p];
    const int64_t kept = kept_bytes(c->ne, c->nv);
    const int64_t span = (c->ne + POOL_ALIGN - 1) / POOL_ALIGN * POOL_ALIGN;
    int64_t alloc = b->alloc + kept;
    int64_t pool_cap = 0, vtx_cap = 0;
    if (P.ra.find(span) < 0) {
        const int64_t old = pool_bytes(p, b->fp32, P.ra.cap);
        // (a capacity whose coefficient arrays pass 2 GiB is never chosen)
        const int64_t max_cap = (int64_t)INT32_MAX / (3 * K_OF[p] * (int64_t)b->w);
        pool_cap = grown_capacity(P.ra.cap, P.ra.cap + span, b->budget - alloc, [&](int64_t nc) {
            return nc <= max_cap ? pool_bytes(p, b->fp32, nc) : INT64_MAX;
        });
        if (pool_cap == 0) return bfail(b, SWE_ENOMEM, "the member does not fit the budget");
        alloc += pool_bytes(p, b->fp32, pool_cap) - old;
    }
    if (b->vra.find(c->nv) < 0) {
        vtx_cap = grown_capacity(b->vra.cap, b->vra.cap + c->nv, b->budget - alloc,
                                 [](int64_t nc) { return 32 * nc; });
        if (vtx_cap == 0) return bfail(b, SWE_ENOMEM, "the member does not fit the budget");
    }
    if (pool_cap) {
        swe_status st = grow_pool(b, p, pool_cap);
        if (st) return st;
    }
    if (vtx_cap) {
        swe_status st = grow_vertices(b, vtx_cap);
        if (st) return st;
    }
    const int64_t first = P.ra.take(span);
    const int64_t vbase = b->vra.take(c->nv);
    if (first < 0 || vbase < 0) {
        if (first >= 0) P.ra.give(first, span);
        if (vbase >= 0) b->vra.give(vbase, c->nv);
        return bfail(b, SWE_ENOMEM, "pool allocation failed");
    }
    const size_t w = b->w, K = c->K;
    BHIP_TRY(b, hipMemcpy2DAsync(static_cast<char *>(P.v.C0) + w * first, w * P.v.cap, c->d_C[0], w * c->stride,
                                 w * c->ne, 3 * K, hipMemcpyDeviceToDevice, b->s));
    BHIP_TRY(b, hipMemcpy2DAsync(static_cast<char *>(P.v.U0) + w * first, w * P.v.cap, c->d_U[0], w * c->stride,
                                 w * c->ne, 2 * K, hipMemcpyDeviceToDevice, b->s));
    BHIP_TRY(b, hipMemcpyAsync(b->d_vtx + vbase, c->d_vtx, sizeof(double4) * c->nv, hipMemcpyDeviceToDevice, b->s));
    BHIP_TRY(b, launch_relocate(c->d_ev, c->d_nb, c->d_nbk, c->d_p, (int)c->ne, c->stride, P.v, (int)first, (int)vbase,
                                b->s));
    const bool no_items = P.v.items != nullptr && !items_cover(c, 0);
    if (P.v.items && items_cover(c, 0))
        BHIP_TRY(b, launch_place_items(c->d_items, c->d_item_off, (int)((c->ne + BLOCK - 1) / BLOCK), P.v, (int)first,
                                       b->s));
    InstDesc &d = b->h_inst[i];
    std::memset(&d, 0, sizeof(d));
    d.first = (int)first;
    d.ne = (int)c->ne;
    d.vbase = (int)vbase;
    d.nv = (int)c->nv;
    d.order = p;
    d.ph.g = c->cfg.g;
    d.ph.fc = c->cfg.f_coriolis;
    d.ph.fric = c->cfg.friction_coef;
    d.ph.friction = c->cfg.friction;
    d.t0 = c->t;
    d.t = c->t;
    d.dt = dt;
    d.steps_left = (int)std::min<int64_t>(nsteps, INT32_MAX);
    d.active = 1;
    d.ncon = c->ncon;
    for (int k = 0; k < c->ncon; ++k) { d.amp[k] = c->amp[k]; d.omega[k] = c->omega[k]; d.phase[k] = c->phase[k]; }
    const bool mixed = !c->uniform || c->cfg.adapt;
    d.mixed = mixed ? 1 : 0;
    d.adapt = c->cfg.adapt ? 1 : 0;
    d.tau = c->cfg.adapt_tau;
    d.p_lo = c->cfg.p_base;
    BHIP_TRY(b, hipMemsetAsync(b->d_flags + i, 0, sizeof(int), b->s));
    swe_status st = put_desc(b, i);
    if (st) return st;
    swe_batch::Member &m = b->mem[i];
    m.ctx = c;
    m.kept = kept;
    m.order = p;
    m.first = first;
    m.span = span;
    m.vbase = vbase;
    m.nv = c->nv;
    m.no_items = no_items;
    m.mixed = mixed;
    m.adapt = c->cfg.adapt != 0;
    if (no_items && b->no_items[p]++ == 0) drop_graph(b);   // the order falls back to the gather kernel
    if (mixed && b->mixed_members[p]++ == 0) drop_graph(b);
    BHIP_TRY(b, hipStreamSynchronize(b->s));   // the copies out of the member's buffers are done
    release_state_buffers(c);
    b->alloc += kept;
    c->batch = b;
    c->slot = i;
    if (per_instance(b, p)) drop_graph(b);   // the step graph launches each such instance
    st = upload_tiles(b);
    if (st) return st;
    *slot = i;
    return SWE_OK;
}

swe_status swe_batch_tick(swe_batch *b, int64_t nsteps)
{
    if (!b || nsteps < 0) return SWE_EINVAL;
    if (nsteps == 0 || swe_batch_resident(b) == 0) return SWE_OK;
    if (!b->gexec) {
        swe_status st = build_step_graph(b);
        if (st) return st;
    }
    for (int64_t k = 0; k < nsteps; ++k) BHIP_TRY(b, hipGraphLaunch(b->gexec, b->s));
    return SWE_OK;
}

swe_status swe_batch_sync(swe_batch *b)
{
    if (!b) return SWE_EINVAL;
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    return SWE_OK;
}

swe_status swe_batch_query(swe_batch *b, int32_t slot, int64_t *steps_left, double *t, int *failed)
{
    if (!b || slot < 0 || slot >= b->cap || !b->mem[slot].ctx) return SWE_EINVAL;
    swe_status st = get_desc(b, slot);
    if (st) return st;
    int f = 0;
    BHIP_TRY(b, hipMemcpyAsync(&f, b->d_flags + slot, sizeof(int), hipMemcpyDeviceToHost, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    if (steps_left) *steps_left = b->h_inst[slot].steps_left;
    if (t) *t = b->h_inst[slot].t;
    if (failed) *failed = f;
    return SWE_OK;
}

swe_status swe_batch_poll(swe_batch *b, int32_t *slots, int32_t *failed, int max, int *n)
{
    if (!b || !slots || !failed || !n || max < 0) return SWE_EINVAL;
    std::vector<int> flags(b->cap);
    BHIP_TRY(b, hipMemcpyAsync(b->h_inst.data(), b->d_inst, sizeof(InstDesc) * b->cap, hipMemcpyDeviceToHost, b->s));
    BHIP_TRY(b, hipMemcpyAsync(flags.data(), b->d_flags, sizeof(int) * b->cap, hipMemcpyDeviceToHost, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    int k = 0;
    for (int i = 0; i < b->cap && k < max; ++i) {
        if (!b->mem[i].ctx) continue;
        if (b->h_inst[i].steps_left <= 0 || flags[i]) {
            slots[k] = i;
            failed[k] = flags[i] ? 1 : 0;
            ++k;
        }
    }
    *n = k;
    return SWE_OK;
}

swe_status swe_batch_retire(swe_batch *b, int32_t slot)
{
    if (!b || slot < 0 || slot >= b->cap || !b->mem[slot].ctx) return SWE_EINVAL;
    swe_batch::Member &m = b->mem[slot];
    swe_ctx *c = m.ctx;
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    swe_status st = get_desc(b, slot);
    if (st) return st;
    st = pull_state(b, slot);
    if (st) return st;
    int f = 0;
    BHIP_TRY(b, hipMemcpyAsync(&f, b->d_flags + slot, sizeof(int), hipMemcpyDeviceToHost, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    c->t = b->h_inst[slot].t;
    if (f) c->failed = true;
    b->h_inst[slot].active = 0;
    b->h_inst[slot].run = 0;
    st = put_desc(b, slot);
    if (st) return st;
    if (per_instance(b, m.order)) drop_graph(b);
    if (m.no_items && --b->no_items[m.order] == 0) drop_graph(b);
    if (m.mixed && --b->mixed_members[m.order] == 0) drop_graph(b);
    const int order = m.order;
    b->pool[order].ra.give(m.first, m.span);
    b->vra.give(m.vbase, m.nv);
    b->alloc -= m.kept;
    m = swe_batch::Member();
    c->batch = nullptr;
    c->slot = -1;
    st = build_items(c);   // the context can step on its own again
    if (st) return bfail(b, st, c->err);
    // an order (or the whole batch) without members holds no pool
    bool any = false, any_order = false;
    for (const auto &q : b->mem) {
        any = any || q.ctx;
        any_order = any_order || (q.ctx && q.order == order);
    }
    if (!any_order) release_pool(b, order);
    if (!any) release_vertices(b);
    return upload_tiles(b);
}

swe_status swe_batch_tile_config(const swe_batch *b, int p, int *tile, int *grid, int *shared)
{
    if (!b || p < 0 || p > 3) return SWE_EINVAL;
    if (tile) *tile = tile_of(b, p);
    if (grid) *grid = b->pool[p].v.cap > 0 ? tile_grid(b, p, tile_of(b, p)) : 0;
    if (shared) *shared = use_shared(b, p) ? 1 : 0;
    return SWE_OK;
}

swe_status swe_batch_set_tile(swe_batch *b, int p, int tile, int shared)
{
    if (!b || p < 0 || p > 3) return SWE_EINVAL;
    if (shared) {
        if (tile != BLOCK) return bfail(b, SWE_EINVAL, "the shared-flux kernel takes 256-element tiles");
        if (!stage_sh_supported(p, b->fp32))
            return bfail(b, SWE_EUNSUPPORTED, "no shared-flux kernel for this order and precision");
    } else if (tile != 64 && tile != 128 && tile != 256) {
        return bfail(b, SWE_EINVAL, "tile must be 64, 128 or 256 elements");
    }
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    b->tile[p] = tile;
    b->shared[p] = shared != 0;
    b->grid[p] = 0;
    drop_graph(b);
    return upload_tiles(b);
}

swe_status swe_batch_tune(swe_batch *b, int reps)
{
    if (!b || reps <= 0) return SWE_EINVAL;
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    // every resident instance takes part without advancing: stage 1 reads
    // buffer 0 and writes buffer 1 only, so the timing launches leave the
    // state untouched; the clock fields are restored afterwards
    std::vector<InstDesc> saved(b->h_inst);
    std::vector<int> flags(b->cap);
    BHIP_TRY(b, hipMemcpyAsync(flags.data(), b->d_flags, sizeof(int) * b->cap, hipMemcpyDeviceToHost, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    for (int i = 0; i < b->cap; ++i) {
        if (!b->mem[i].ctx) continue;
        swe_status st = get_desc(b, i);
        if (st) return st;
        saved[i] = b->h_inst[i];
        b->h_inst[i].run = 1;
        st = put_desc(b, i);
        if (st) return st;
    }
    hipEvent_t e0, e1;
    BHIP_TRY(b, hipEventCreate(&e0));
    BHIP_TRY(b, hipEventCreate(&e1));
    // candidates: the gather kernel with tiles of 64, 128 or 256 elements,
    // and (orders with edge items) the shared-flux kernel on 256-element tiles
    const int tiles[4] = {64, 128, 256, BLOCK};
    swe_status st = SWE_OK;
    for (int p = 0; p < 4 && st == SWE_OK; ++p) {
        bool any = false;
        for (int i = 0; i < b->cap; ++i) any = any || (b->mem[i].ctx && b->mem[i].order == p);
        if (!any || per_instance(b, p)) continue;
        float best = 1e30f;
        int bt = b->tile[p], bg = b->grid[p];
        bool bs = b->shared[p];
        for (int ti = 0; ti < 4 && st == SWE_OK; ++ti) {
            const bool sh = ti == 3;
            b->tile[p] = tiles[ti];
            b->shared[p] = sh;
            if (sh && !use_shared(b, p)) continue;
            st = upload_tiles(b);
            if (st) break;
            const int grid = tile_grid(b, p, tiles[ti]);
            Sink k;
            k.s = b->s;
            auto launch = [&]() {
                return sh ? launch_batch_stage_sh(p, b->fp32, MODE_STAGE1, batch_args(b, p), grid, k)
                          : launch_batch_stage(p, b->fp32, MODE_STAGE1, tiles[ti], batch_args(b, p), grid, k);
            };
            hipError_t e = launch();
            if (e == hipSuccess) e = hipEventRecord(e0, b->s);
            for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch();
            if (e == hipSuccess) e = hipEventRecord(e1, b->s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                st = bfail(b, SWE_EDEVICE, std::string("tuning: ") + hipGetErrorString(e));
                break;
            }
            if (ms < best) { best = ms; bt = tiles[ti]; bg = grid; bs = sh; }
        }
        b->shared[p] = bs;
        b->tile[p] = bt;
        b->grid[p] = bg;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    for (int i = 0; i < b->cap; ++i) {
        if (!b->mem[i].ctx) continue;
        b->h_inst[i] = saved[i];
        swe_status s2 = put_desc(b, i);
        if (st == SWE_OK) st = s2;
    }
    // stage 1 also checked depths: the flags go back to what the real run had
    BHIP_TRY(b, hipMemcpyAsync(b->d_flags, flags.data(), sizeof(int) * b->cap, hipMemcpyHostToDevice, b->s));
    BHIP_TRY(b, hipStreamSynchronize(b->s));
    if (st == SWE_OK) st = upload_tiles(b);
    drop_graph(b);
    return st;
}

}  // extern "C"
