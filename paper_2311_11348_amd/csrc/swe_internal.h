// Internal interface between the host runtime (swe_api.cpp) and the gfx950
// kernels (swe_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace swe {

constexpr int KMAX = 10;
constexpr int BLOCK = 256;
constexpr int NCON_MAX = 16;

// Boundary codes stored in the neighbour array in place of an element id.
constexpr int NB_LAND = -1;
constexpr int NB_OPEN = -2;

// An empty slot in a block's list of edge items of the shared-flux kernels
// (it aligns the next kind of item to a wave of 64 lanes).
constexpr unsigned ITEM_PAD = 0xffffffffu;

enum StageMode { MODE_RHS = 0, MODE_STAGE1 = 1, MODE_STAGE2 = 2 };

struct Physics {
    double g;
    double fc;
    double fric;      // kappa (linear) or C_f (quadratic)
    int friction;     // 0 none, 1 linear, 2 quadratic
};

// Device view of one mesh and its fields.  Element-indexed arrays use a
// structure-of-arrays layout [slot][stride] with stride >= ne, a multiple of
// the block size; coefficient arrays are [component][mode][stride] with
// KS stored modes per component, in reference-scaled form (coefficient of
// the reference-element basis, i.e. physical coefficient / sqrt(|det B_e|)).
struct MeshView {
    int ne;
    int stride;
    int KS;                               // stored modes per component
    const double4 *__restrict__ vtx;      // (x, y, h_b, 0) per vertex
    const int *__restrict__ ev;           // [3][stride] vertex ids, counter-clockwise
    const int *__restrict__ enb;          // [3][stride] neighbour id or NB_LAND / NB_OPEN
    const unsigned char *__restrict__ enbk;  // [stride] neighbour's local edge, 2 bits per edge
    const signed char *__restrict__ ep;   // [stride] element order (may be null if uniform)
};

template <typename Real>
struct StageArgs {
    MeshView m;
    const Real *Cin;     // stage input state c^(s)
    const Real *Uin;     // velocity of c^(s)
    const Real *Cn;      // c^n for the second stage (may alias Cout)
    Real *Cout;
    Real *Uout;
    Real *Lout;          // MODE_RHS output
    const Real *src;     // optional extra right-hand side (reference-scaled), or null
    Physics ph;
    double xihat;        // open-boundary elevation at the stage time
    double dt;
    int *flag;           // set to 1 on a non-finite value or non-positive mean depth
    int mixed;           // element orders differ: mask modes above K(p_e)
    // order-separated scheme
    unsigned char *inlist;         // [stride] 1 if the element has a correction
    Real *Lb;            // [3][K(p_base)][stride] base partial stage values of listed elements
    Real *Lc;            // [3][KS][stride] dt * correction of listed elements
    int finish;          // correction kernel: 0 leaves dt * correction in Lc for the
                         // epilogue; MODE_STAGE1 / MODE_STAGE2 joins it with the base
                         // part in Lb and finishes the listed element's stage itself
    const int *list;     // listed elements of one order
    const int *count;    // device-side length of list
    int *listw;          // [4][lcap] lists being rebuilt by the order update
    int *cntw;           // [4] their lengths
    Real *Calt, *Ualt;   // the other state/velocity buffer (order update clears dropped modes)
    // batched instance launched on its own: element indices start at e_off in
    // the pooled arrays; step, open-sea elevation and run flag come from inst
    const struct InstDesc *inst;
    int e_off;
    int stage;           // with inst: which stage time of the step (0 or 1) a kernel without MODE uses
    int skip_listed;     // base kernel of the order-partitioned scheme: listed elements are not its work
    int blocks;          // stage launchers: cover the first blocks * BLOCK elements only (0: all)
};

struct InstDesc;

// One resident instance of a batch.  Its elements occupy [first, first + ne)
// of the pool of its order and its vertices [vbase, vbase + nv) of the vertex
// pool; neighbour and vertex ids in the pools are already offset.
struct InstDesc {
    int first, ne, vbase, nv;
    int order;
    int active, run;             // resident / advancing in the current step
    int steps_done, steps_left;
    int ncon;
    int mixed;                   // per-element orders (pool ep) mask the stage
    int adapt;                   // orders re-chosen by the indicator before every step
    int p_lo;                    // lowest order of an indicator-driven member (its base order)
    Physics ph;
    double tau;                  // indicator threshold of an indicator-driven member
    double t0, t, dt;            // start time, current time, step
    double xh[2];                // open-sea elevation at the two stage times of this step
    double amp[4], omega[4], phase[4];
};

// Pooled arrays of one order class (structure of arrays, stride cap).
struct PoolView {
    void *C0, *C1, *U0, *U1;     // state and velocity ping-pong buffers [slot][cap]
    int *ev, *nb;                // [3][cap]
    unsigned char *nbk;          // [cap]
    unsigned *items;             // edge items of the shared-flux kernel, 3 slots per element:
                                 // the block at element f (f a multiple of 256) keeps its items from 3 f
    int *nitems;                 // [cap / 256] item count of each 256-element block
    signed char *ep;             // [cap] element orders (uniform members: their order)
    signed char *pnew;           // [cap] orders chosen by the indicator, before they are applied
    int cap;
};

struct BatchArgs {
    PoolView pool;               // pool of the launched order
    const double4 *vtx;          // vertex pool
    const InstDesc *inst;
    const int2 *tiles;           // [tile_cap] (instance, first element) of the launched order
    const int *ntiles;           // device-side tile count of the launched order
    const int2 *atiles;          // 256-element tiles of the launched order's indicator-driven members
    const int *natiles;          // their device-side count
    int *flags;                  // [instances]
};

// Launchers (defined in swe_kernels.hip).  Return hipSuccess or the launch error.
// Where a launch goes: a stream, or (g set) a kernel node appended to a graph
// under construction, after the node appended before it.  Graphs built this
// way need no stream capture, so other host threads may keep calling HIP
// (allocations, copies) while a step graph is being built.
struct Sink {
    hipStream_t s = nullptr;
    hipGraph_t g = nullptr;
    static constexpr int MAXDEP = 6;
    hipGraphNode_t dep[MAXDEP] = {};   // what the next node waits for
    int ndep = 0;
    // the next node also waits for what another branch ended with (a join)
    bool join(const Sink &o)
    {
        for (int i = 0; i < o.ndep; ++i) {
            bool have = false;
            for (int j = 0; j < ndep; ++j) have = have || dep[j] == o.dep[i];
            if (have) continue;
            if (ndep == MAXDEP) return false;
            dep[ndep++] = o.dep[i];
        }
        return true;
    }
};
hipError_t emit(Sink &k, const void *fn, dim3 grid, dim3 block, void **args);

hipError_t launch_stage(int p, bool fp32, int mode, bool sep, const void *args, hipStream_t s);
hipError_t launch_stage(int p, bool fp32, int mode, bool sep, const void *args, Sink &k);
// fused stage with each in-block edge flux computed once (edge items built by
// the host, see swe_kernels.hip); used for p = 1 to 3
bool stage_sh_supported(int p, bool fp32);
hipError_t launch_stage_sh(int p, bool fp32, int mode, const void *args, const unsigned *items, const int *item_off,
                           Sink &k);
// The listed elements of every order in one launch (orders lo..pn, nblk
// blocks per order; lists at args.list + p * lcap, lengths args.count[p]):
// full stage (order-partitioned scheme), correction and epilogue (order-
// separated scheme, lo = b)
hipError_t launch_full_all(int lo, int pn, bool fp32, int mode, const void *args, int nblk, int lcap, Sink &k);
hipError_t launch_corr_all(int b, int pn, bool fp32, const void *args, double dt, int nblk, int lcap, Sink &k);
hipError_t launch_epi_all(int b, int pn, bool fp32, int mode, const void *args, int nblk, int lcap, Sink &k);
// The correction of the order-separated scheme for the listed elements
// [e0, e1) on nthreads host threads (args: host copies of mesh, state and
// Lc; order: host element orders); the same element code as the GPU's.
// Returns 0, or -1 for an unsupported (b, pn).
int host_corr(int b, int pn, bool fp32, const void *args, double dt, const signed char *order, int e0, int e1,
              int nthreads);
hipError_t launch_usolve(int p, bool fp32, const void *args, hipStream_t s);
// minimum depth control over every element of the stage output (args.Cout,
// args.Uout; per-element orders from args.m.ep, at most pm)
hipError_t launch_depth_limit(int pm, bool fp32, const void *args, double h_min, Sink &k);
hipError_t launch_indicator(bool fp32, const void *args, double tau, int p_lo, int p_hi, double *I_out,
                            signed char *p_new, Sink &k);
// clock (or null): the instance whose step clock advances in the same launch
// (a step graph's order update; see k_batch_clock), flag its failure flag
hipError_t launch_apply_order(int pm, bool fp32, const void *args, const signed char *p_new, signed char *p_cur,
                              int p_base, int lcap, InstDesc *clock, const int *flag, Sink &k);
hipError_t launch_indicator(bool fp32, const void *args, double tau, int p_lo, int p_hi, double *I_out,
                            signed char *p_new, hipStream_t s);
hipError_t launch_mass(const MeshView &m, bool fp32, const void *C, double *partial,
                       double *out, hipStream_t s);
// The same reduction with its partial sums in a fixed device array of
// MASS_SCRATCH_PARTIALS doubles (ne <= MASS_SCRATCH_PARTIALS * BLOCK), no
// allocation; the result goes to the device pointer out.
constexpr int MASS_SCRATCH_PARTIALS = 16384;
hipError_t launch_mass_noalloc(const MeshView &m, bool fp32, const void *C, double *out, hipStream_t s);
// Device address of that array on the current device (resolved once per
// device, kept for the process); out may be null.
hipError_t mass_scratch(double **out);
int mass_partials(int ne);
hipError_t launch_batch_stage(int p, bool fp32, int mode, int tile, const BatchArgs &b, int grid, Sink &k);
hipError_t launch_batch_clock(InstDesc *inst, const int *flags, int n, Sink &k);
// write one instance descriptor in stream order (no host buffer outlives the call)
hipError_t launch_inst_set(InstDesc *inst, const InstDesc &v, hipStream_t s);
// copy an instance's mesh arrays into a pool, offsetting vertex and element ids
// batched shared-flux stage (one 256-element tile per block; orders with
// stage_sh_supported); items placed in the pool by launch_place_items
hipError_t launch_batch_stage_sh(int p, bool fp32, int mode, const BatchArgs &b, int grid, Sink &k);
hipError_t launch_place_items(const unsigned *items, const int *item_off, int nblk, const PoolView &pool, int first,
                              hipStream_t s);
hipError_t launch_relocate(const int *ev, const int *nb, const unsigned char *nbk, const signed char *ep, int ne,
                           int stride, const PoolView &pool, int first, int vbase, hipStream_t s);
// order update of a batch's indicator-driven members of one order class:
// indicator into pool.pnew, then the new orders applied (fused scheme, no lists)
hipError_t launch_batch_indicator(bool fp32, const BatchArgs &b, int grid, Sink &k);
hipError_t launch_batch_apply(int pm, bool fp32, const BatchArgs &b, int grid, Sink &k);

}  // namespace swe
