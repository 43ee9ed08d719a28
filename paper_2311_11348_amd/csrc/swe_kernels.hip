// gfx950 kernels of the quadrature-free DG shallow-water right-hand side.
//
// One thread owns one element.  Per stage it
//   1. rebuilds the element geometry from its three vertices (FP64),
//   2. evaluates the volume term (A, grad phi) of (variational_disc_1) as
//      contractions with the exact basis-product tensors: the flux products
//      are projected onto P^{p-1} with C[m][i][j] and mapped back with the
//      derivative matrix D[k][q][m] (eq. (mass_basis) for the mass row, the
//      same tensor algebra for the momentum rows),
//   3. adds the source (r, phi) of (def_A_h_qf),
//   4. gathers its three edges: traces of both sides in 1D Legendre modes,
//      Lax-Friedrichs flux with the constant-part penalty (eq:lambda), 1D
//      triple products G for the flux products, and the trace matrix R to
//      test against its own basis,
//   5. combines the SSP-RK2 stage and solves u H = q (variational_disc_2) for
//      the new state with the truncated depth expansion K(p,i,j) of
//      Sec. "order separation", by LDL^T in registers.
//
// Coefficients are reference-scaled: c_hat = c / sqrt(|det B_e|), which makes
// every tensor contraction independent of the element size; only the inverse
// Jacobian, the edge normals and |E|/|det B_e| enter.  Terms carrying the
// bathymetry (well-balancing: g xi h_b in the flux, g xi grad h_b in the
// source) are always accumulated in FP64.
//
// Kernel families below: the element-gather stage above (k_stage); the
// shared-flux stage (k_stage_sh, stage_sh_block), where each edge flux
// inside a block of 256 elements is computed once from host-built edge
// items and handed to both sides through LDS; the listed elements of the
// order-separated and order-partitioned schemes (k_corr_all, k_full_all,
// k_epi_all), by teams of four waves per 64 entries or one element per
// thread, with the correction kernel doing the epilogue's join itself when
// it runs after the base pass in one chain; the order update (k_indicator,
// k_apply_order); the batch forms of the stage and order update; the
// minimum depth control; the FP64 mass reduction.
#include "swe_internal.h"
#include "swe_tables.h"

#include <algorithm>
#include <mutex>
#include <thread>
#include <type_traits>
#include <vector>

namespace swe {
namespace {

constexpr double TC[10][10][10] = SWET_C;
constexpr double TD[2][10][10] = SWET_D;
constexpr double TR[3][10][4] = SWET_R;
constexpr double TG[4][4][4] = SWET_G;
constexpr double TW[3][3] = SWET_W;
constexpr double TPMID[3][3] = SWET_PMID;
constexpr double TCHK[6][10] = SWET_PCHK;
constexpr int TDEG[10] = SWET_DEG;
constexpr int KOFP[4] = SWET_K_OF_P;
constexpr double SQRT2 = 1.41421356237309504880;
constexpr double INV_2SQRT3 = 0.28867513459481288225;  // 1 / (2 sqrt 3)

// Minimum resident waves per SIMD the register allocator must allow for the
// stage kernel (more waves hide memory latency; fewer avoid spills).
#ifndef SWE_WAVES_FP64
#define SWE_WAVES_FP64 1
#endif
#ifndef SWE_WAVES_FP32
#define SWE_WAVES_FP32 2
#endif
#ifndef SWE_WAVES_FP32_P3
#define SWE_WAVES_FP32_P3 1
#endif
template <int P, typename Real>
constexpr int waves_target()
{
    // Order 3 needs more than 256 registers per lane: one wave (the
    // accumulation registers then serve as spill space; no kernel loops
    // around such an evaluation, which gave run-to-run differences).
    return P >= 3 ? (std::is_same<Real, double>::value ? 1 : SWE_WAVES_FP32_P3)
                  : P <= 1 ? 2 : (std::is_same<Real, double>::value ? SWE_WAVES_FP64 : SWE_WAVES_FP32);
}

template <int P>
struct Ord {
    static constexpr int K = (P + 1) * (P + 2) / 2;   // modes of P^p
    static constexpr int KM = P * (P + 1) / 2;        // modes of P^{p-1}
    static constexpr int NT = P + 1;                  // Legendre modes of a trace
};

__device__ __forceinline__ int xcd_block(int b, int nb)
{
    // Workgroups are dispatched round-robin over the 8 XCDs.  Give each XCD a
    // contiguous range of element tiles so that neighbour gathers hit its L2.
    const int q = nb >> 3, r = nb & 7;
    const int x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// The element code below is compiled for the host as well: the order-separated
// scheme's correction can run on the CPU beside the GPU's base pass (the
// heterogeneous stage).  Only the element-indexed loads and stores differ.
#define SWE_HD __host__ __device__ __forceinline__

template <typename T>
SWE_HD T tmax(T a, T b) { return a > b ? a : b; }

// FP32 reciprocal and square root by the hardware's single-instruction
// approximations (about 1 ulp) instead of the correctly rounded sequences
// (ten and more instructions each).  Used on FP32 data only, where the
// argument is a positive, well-scaled quantity: the pivots of the depth
// matrix H, the squared wave speed of the penalty, the squared velocity of
// the quadratic friction.  The host build (the heterogeneous stage) rounds
// correctly.
SWE_HD float rcp_approx(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_rcpf(x);
#else
    return 1.0f / x;
#endif
}

SWE_HD float sqrt_approx(float x)
{
#if defined(__HIP_DEVICE_COMPILE__)
    return __builtin_amdgcn_sqrtf(x);
#else
    return std::sqrt(x);
#endif
}

// Element-indexed arrays are read and written through buffer resources: a
// uniform descriptor (base, byte size) in scalar registers, a uniform byte
// offset per (component, mode) slot and one 32-bit lane offset, so no load
// needs per-lane 64-bit address arithmetic, and an access beyond the array
// (which the host never issues) reads 0 instead of faulting.
constexpr int RSRC_WORD3 = 0x00020000;   // raw 32-bit access, gfx9 family
typedef unsigned int u32x2 __attribute__((__vector_size__(8)));
// cache-policy operand of a buffer access: the non-temporal bit (gfx94x/gfx950)
constexpr int CPOL_NT = 2;

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void *p, unsigned bytes)
{
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), (short)0, (int)bytes, RSRC_WORD3);
}

template <typename T>
struct Buf {
#if defined(__HIP_DEVICE_COMPILE__)
    __amdgpu_buffer_rsrc_t r;
#else
    // on the host: the array and its size, with the same out-of-range
    // behaviour (loads read 0, stores are dropped)
    char *base;
    unsigned size;
#endif
    int slot_bytes;
    SWE_HD Buf(const T *p, int nslots, int stride)
#if defined(__HIP_DEVICE_COMPILE__)
        : r(make_rsrc(p, (unsigned)nslots * (unsigned)stride * (unsigned)sizeof(T))),
#else
        : base(reinterpret_cast<char *>(const_cast<T *>(p))),
          size((unsigned)nslots * (unsigned)stride * (unsigned)sizeof(T)),
#endif
          slot_bytes(stride * (int)sizeof(T)) {}
    // off = element index * sizeof(T)
    SWE_HD T ld(int slot, unsigned off) const
    {
#if defined(__HIP_DEVICE_COMPILE__)
        if constexpr (sizeof(T) == 8)
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)off, slot * slot_bytes, 0));
        else
            return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)off, slot * slot_bytes, 0));
#else
        const unsigned at = off + (unsigned)(slot * slot_bytes);
        if (!base || at + sizeof(T) > size) return T(0);
        T v;
        __builtin_memcpy(&v, base + at, sizeof(T));
        return v;
#endif
    }
    // a store that is not kept in the caches (the non-temporal policy bit):
    // for results no block of the same launch reads back
    SWE_HD void st_stream(int slot, unsigned off, T v) const
    {
#if defined(__HIP_DEVICE_COMPILE__)
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off,
                                                  slot * slot_bytes, CPOL_NT);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off,
                                                  slot * slot_bytes, CPOL_NT);
#else
        st(slot, off, v);
#endif
    }
    SWE_HD void st(int slot, unsigned off, T v) const
    {
#if defined(__HIP_DEVICE_COMPILE__)
        if constexpr (sizeof(T) == 8)
            __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)off,
                                                  slot * slot_bytes, 0);
        else
            __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, (int)off,
                                                  slot * slot_bytes, 0);
#else
        const unsigned at = off + (unsigned)(slot * slot_bytes);
        if (base && at + sizeof(T) <= size) __builtin_memcpy(base + at, &v, sizeof(T));
#endif
    }
};

struct Geo {
    double b00, b01, b10, b11;   // inverse Jacobian: d(xh)/dx, d(xh)/dy, d(yh)/dx, d(yh)/dy
    double det;                  // |det B_e| = 2 area
    double idet;                 // 1 / |det B_e|
    double X[3], Y[3], h[3];     // vertices and depths
};

// Geometry from the element's vertex ids (already loaded).
SWE_HD void geo_from_ids(const double4 *vtx, const int (&id3)[3], Geo &G)
{
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const double4 p = vtx[(unsigned)id3[v]];
        G.X[v] = p.x;
        G.Y[v] = p.y;
        G.h[v] = p.z;
    }
    const double a00 = G.X[1] - G.X[0], a01 = G.X[2] - G.X[0];
    const double a10 = G.Y[1] - G.Y[0], a11 = G.Y[2] - G.Y[0];
    G.det = a00 * a11 - a01 * a10;
    const double id = 1.0 / G.det;
    G.idet = id;
    G.b00 = a11 * id;
    G.b01 = -a01 * id;
    G.b10 = -a10 * id;
    G.b11 = a00 * id;
}

SWE_HD void load_geo(const double4 *vtx, const Buf<int> &ev, unsigned offi, Geo &G)
{
#pragma unroll
    for (int v = 0; v < 3; ++v) {
        const double4 p = vtx[(unsigned)ev.ld(v, offi)];
        G.X[v] = p.x;
        G.Y[v] = p.y;
        G.h[v] = p.z;
    }
    const double a00 = G.X[1] - G.X[0], a01 = G.X[2] - G.X[0];
    const double a10 = G.Y[1] - G.Y[0], a11 = G.Y[2] - G.Y[0];
    G.det = a00 * a11 - a01 * a10;
    const double id = 1.0 / G.det;
    G.idet = id;
    G.b00 = a11 * id;
    G.b01 = -a01 * id;
    G.b10 = -a10 * id;
    G.b11 = a00 * id;
}

template <int P, typename Real>
struct Fields {
    static constexpr int K = Ord<P>::K;
    Real xi[K], U[K], V[K], u[K], v[K];
};

template <int P, typename Real>
SWE_HD void load_state(const Buf<Real> &C, const Buf<Real> &Uv, int KS, unsigned off,
                                           Fields<P, Real> &s)
{
    constexpr int K = Ord<P>::K;
#pragma unroll
    for (int i = 0; i < K; ++i) {
        s.xi[i] = C.ld(0 * KS + i, off);
        s.U[i] = C.ld(1 * KS + i, off);
        s.V[i] = C.ld(2 * KS + i, off);
        s.u[i] = Uv.ld(0 * KS + i, off);
        s.v[i] = Uv.ld(1 * KS + i, off);
    }
}

// t_i = sum_j C[m][i][j] g_j with the zero pattern folded at compile time
template <int K, typename T, typename S>
SWE_HD T crow(int m, int i, const S (&g)[K])
{
    T t = T(0);
#pragma unroll
    for (int j = 0; j < K; ++j)
        if (TC[m][i][j] != 0.0) t = fma(T(TC[m][i][j]), T(g[j]), t);
    return t;
}

template <int K>
SWE_HD constexpr bool crow_nonzero(int m, int i)
{
    bool any = false;
    for (int j = 0; j < K; ++j) any = any || (TC[m][i][j] != 0.0);
    return any;
}

// ------------------------------------------------------------ accumulator
// acc = c + dt * L(c), built term by term (every geometric factor carries dt).
// Bathymetry terms go to W: FP64 always; for Real = double W is the momentum
// rows of L itself, for Real = float a separate FP64 array added at the end.
template <int P, typename Real>
struct Acc {
    static constexpr int K = Ord<P>::K;
    static constexpr bool SPLIT = !std::is_same<Real, double>::value;
    Real L[3][K];
    double W[SPLIT ? 2 : 1][SPLIT ? K : 1];
    SWE_HD double &w(int j, int q)
    {
        if constexpr (SPLIT) return W[j][q];
        else return L[1 + j][q];
    }
};

// ------------------------------------------------------------ volume term
// acc[j][q] += dt sum_k sum_m D[k][q][m] (Bi_kx F^j_x,m + Bi_ky F^j_y,m), over the
// projected modes M0 <= m < M1 (all of them by default)
template <int P, typename Real, int M0 = 0, int M1 = Ord<P>::KM>
SWE_HD void volume_term(const Fields<P, Real> &s, const double (&hbh)[3],
                                            const Geo &G, double g, double dt, Acc<P, Real> &A)
{
    constexpr int K = Ord<P>::K, KM = Ord<P>::KM;
    if constexpr (KM > 0 && M0 < M1) {
        Real Fx[3][KM], Fy[3][KM];
        double FW[KM];
        const Real hg = Real(0.5 * g);
#pragma unroll
        for (int m = M0; m < M1; ++m) {
            Real pUu = 0, pUv = 0, pVu = 0, pVv = 0, pxx = 0;
            double pxh = 0.0;
#pragma unroll
            for (int i = 0; i < K; ++i) {
                if (!crow_nonzero<K>(m, i)) continue;
                const Real tu = crow<K, Real>(m, i, s.u);
                const Real tv = crow<K, Real>(m, i, s.v);
                const Real tx = crow<K, Real>(m, i, s.xi);
                pUu = fma(s.U[i], tu, pUu);
                pUv = fma(s.U[i], tv, pUv);
                pVu = fma(s.V[i], tu, pVu);
                pVv = fma(s.V[i], tv, pVv);
                pxx = fma(s.xi[i], tx, pxx);
                double th = 0.0;
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    if (TC[m][i][j] != 0.0) th = fma(TC[m][i][j], hbh[j], th);
                pxh = fma(double(s.xi[i]), th, pxh);
            }
            Fx[0][m] = s.U[m];
            Fy[0][m] = s.V[m];
            Fx[1][m] = fma(hg, pxx, pUu);
            Fy[1][m] = pUv;
            Fx[2][m] = pVu;
            Fy[2][m] = fma(hg, pxx, pVv);
            FW[m] = g * dt * pxh;
        }
        const Real b00 = Real(G.b00 * dt), b01 = Real(G.b01 * dt);
        const Real b10 = Real(G.b10 * dt), b11 = Real(G.b11 * dt);
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            Real G0[KM], G1[KM];
#pragma unroll
            for (int m = M0; m < M1; ++m) {
                G0[m] = fma(b00, Fx[j][m], b01 * Fy[j][m]);
                G1[m] = fma(b10, Fx[j][m], b11 * Fy[j][m]);
            }
#pragma unroll
            for (int q = 0; q < K; ++q) {
                Real acc = A.L[j][q];
#pragma unroll
                for (int m = M0; m < M1; ++m) {
                    if (TD[0][q][m] != 0.0) acc = fma(Real(TD[0][q][m]), G0[m], acc);
                    if (TD[1][q][m] != 0.0) acc = fma(Real(TD[1][q][m]), G1[m], acc);
                }
                A.L[j][q] = acc;
            }
        }
        // bathymetry part of the pressure: x-momentum uses Bi_kx, y-momentum Bi_ky
        double Wx[KM], Wy[KM], Zx[KM], Zy[KM];
#pragma unroll
        for (int m = M0; m < M1; ++m) {
            Wx[m] = G.b00 * FW[m];
            Wy[m] = G.b01 * FW[m];
            Zx[m] = G.b10 * FW[m];
            Zy[m] = G.b11 * FW[m];
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            double ax = A.w(0, q), ay = A.w(1, q);
#pragma unroll
            for (int m = M0; m < M1; ++m) {
                if (TD[0][q][m] != 0.0) {
                    ax = fma(TD[0][q][m], Wx[m], ax);
                    ay = fma(TD[0][q][m], Wy[m], ay);
                }
                if (TD[1][q][m] != 0.0) {
                    ax = fma(TD[1][q][m], Zx[m], ax);
                    ay = fma(TD[1][q][m], Zy[m], ay);
                }
            }
            A.w(0, q) = ax;
            A.w(1, q) = ay;
        }
    }
}

// ------------------------------------------------------------ source term
template <int P, typename Real>
SWE_HD void source_term(const Fields<P, Real> &s, const Geo &G, const Physics &ph,
                                            double dt, Acc<P, Real> &A)
{
    constexpr int K = Ord<P>::K;
    const double dh1 = G.h[1] - G.h[0], dh2 = G.h[2] - G.h[0];
    const double gx = ph.g * dt * (G.b00 * dh1 + G.b10 * dh2);   // dt g dh_b/dx
    const double gy = ph.g * dt * (G.b01 * dh1 + G.b11 * dh2);   // dt g dh_b/dy
    const Real fc = Real(ph.fc * dt);
    Real tau = 0;
    if (ph.friction == 2) {
        // |constant part of u| = sqrt(2) |(u_0, v_0)| in reference-scaled modes
        const Real um = s.u[0], vm = s.v[0];
        if constexpr (std::is_same<Real, double>::value)
            tau = Real(ph.fric * dt * SQRT2) * sqrt(um * um + vm * vm);
        else
            tau = Real(ph.fric * dt * SQRT2) * sqrt_approx(um * um + vm * vm);
    } else if (ph.friction == 1) {
        tau = Real(ph.fric * dt);
    }
#pragma unroll
    for (int q = 0; q < K; ++q) {
        Real a1 = fma(fc, s.V[q], A.L[1][q]);
        Real a2 = fma(-fc, s.U[q], A.L[2][q]);
        if (ph.friction == 2) {
            a1 = fma(-tau, s.u[q], a1);
            a2 = fma(-tau, s.v[q], a2);
        } else if (ph.friction == 1) {
            a1 = fma(-tau, s.U[q], a1);
            a2 = fma(-tau, s.V[q], a2);
        }
        A.L[1][q] = a1;
        A.L[2][q] = a2;
        A.w(0, q) = fma(gx, double(s.xi[q]), A.w(0, q));
        A.w(1, q) = fma(gy, double(s.xi[q]), A.w(1, q));
    }
}

// ------------------------------------------------------------ edge terms
// trace on a local edge in Legendre modes: t_a = sum_n f_n R[k][n][a]
template <int P, typename Real>
SWE_HD void trace_own(int k, const Real (&f)[Ord<P>::K], Real (&t)[Ord<P>::NT])
{
    constexpr int K = Ord<P>::K, NT = Ord<P>::NT;
#pragma unroll
    for (int a = 0; a < NT; ++a) {
        Real acc = 0;
#pragma unroll
        for (int n = 0; n < K; ++n)
            if (TR[k][n][a] != 0.0) acc = fma(f[n], Real(TR[k][n][a]), acc);
        t[a] = acc;
    }
}

// 1D product projected onto Legendre modes c <= P: out_c = sum_ab G[c][a][b] f_a g_b
template <int NT, typename T>
SWE_HD T prod1(int c, const T (&f)[NT], const T (&g)[NT])
{
    T acc = 0;
#pragma unroll
    for (int a = 0; a < NT; ++a) {
        T t = 0;
        bool any = false;
#pragma unroll
        for (int b = 0; b < NT; ++b)
            if (TG[c][a][b] != 0.0) {
                t = fma(T(TG[c][a][b]), g[b], t);
                any = true;
            }
        if (any) acc = fma(f[a], t, acc);
    }
    return acc;
}

// Edge terms of one element of order P whose neighbours have order <= PN
// (their stored modes above their own order are zero).  Both traces are
// expanded to NX = max(P, PN) + 1 Legendre modes; the flux is projected onto
// the own test space (modes <= P).
// The edge term of local edge k (its flux lifted onto the element's modes).
template <int P, int PN, typename Real, int k>
SWE_HD void edge_one(const MeshView &m, unsigned e, const Buf<Real> &bC, const Buf<Real> &bU,
                     const Buf<int> &bNb, const Fields<P, Real> &s, const Geo &G, double g, double xihat,
                     double dt, const Real (*sR)[Ord<PN>::K][(P > PN ? P : PN) + 1], Acc<P, Real> &A)
{
    constexpr int K = Ord<P>::K, NT = Ord<P>::NT, KN = Ord<PN>::K;
    constexpr int NX = (P > PN ? P : PN) + 1;
    const int KS = m.KS;
    const unsigned nbk_all = m.enbk[e];
    const Real xbm = Real(SQRT2) * s.xi[0];
    const Real ubm = Real(SQRT2) * s.u[0], vbm = Real(SQRT2) * s.v[0];
    // With the edge vector's normal nu = |E| n (no square root), every flux
    // term carries |E| n or |E| lambda, and |E| / |det B| folds into dt / |det B|.
    const double dt_det = dt * G.idet;
    {
        constexpr int ka = (k + 1) % 3, kb = (k + 2) % 3;
        const double dx = G.X[kb] - G.X[ka], dy = G.Y[kb] - G.Y[ka];
        const double len2 = dx * dx + dy * dy;
        const Real nx = Real(dy), ny = Real(-dx);          // |E| n
        const double hmid = 0.5 * (G.h[ka] + G.h[kb]);
        const double hbt[2] = {hmid, (G.h[kb] - G.h[ka]) * INV_2SQRT3};

        Real txm[NX], tUm[NX], tVm[NX], unm[NX], qnm[NX];
        {
            Real tx[NT], tU[NT], tV[NT], tu[NT], tv[NT];
            trace_own<P, Real>(k, s.xi, tx);
            trace_own<P, Real>(k, s.U, tU);
            trace_own<P, Real>(k, s.V, tV);
            trace_own<P, Real>(k, s.u, tu);
            trace_own<P, Real>(k, s.v, tv);
#pragma unroll
            for (int a = 0; a < NT; ++a) {
                txm[a] = tx[a];
                tUm[a] = tU[a];
                tVm[a] = tV[a];
                unm[a] = fma(tu[a], nx, tv[a] * ny);
                qnm[a] = fma(tU[a], nx, tV[a] * ny);
            }
#pragma unroll
            for (int a = NT; a < NX; ++a) {
                txm[a] = 0; tUm[a] = 0; tVm[a] = 0; unm[a] = 0; qnm[a] = 0;
            }
        }

        const int nb = bNb.ld(k, e * 4u);
        Real txp[NX], tUp[NX], tVp[NX], unp[NX], qnp[NX];
        Real xbp, unbp;
        const Real unbm = fabs(fma(ubm, nx, vbm * ny));
        if (nb >= 0) {
            const int kk = (nbk_all >> (2 * k)) & 3;
            Real tup[NX], tvp[NX];
#pragma unroll
            for (int a = 0; a < NX; ++a) {
                txp[a] = 0; tUp[a] = 0; tVp[a] = 0; tup[a] = 0; tvp[a] = 0;
            }
            const unsigned un_ = (unsigned)nb * (unsigned)sizeof(Real);
            Real x0 = 0, u0 = 0, v0 = 0;
#pragma unroll
            for (int n = 0; n < KN; ++n) {
                const Real fx = bC.ld(0 * KS + n, un_);
                const Real fU = bC.ld(1 * KS + n, un_);
                const Real fV = bC.ld(2 * KS + n, un_);
                const Real fu = bU.ld(0 * KS + n, un_);
                const Real fv = bU.ld(1 * KS + n, un_);
                if (n == 0) { x0 = fx; u0 = fu; v0 = fv; }
                // the trace of a degree-d basis function has no Legendre mode above d
#pragma unroll
                for (int a = 0; a < NX && a <= TDEG[n]; ++a) {
                    const Real r = sR[kk][n][a];
                    txp[a] = fma(fx, r, txp[a]);
                    tUp[a] = fma(fU, r, tUp[a]);
                    tVp[a] = fma(fV, r, tVp[a]);
                    tup[a] = fma(fu, r, tup[a]);
                    tvp[a] = fma(fv, r, tvp[a]);
                }
            }
            // the neighbour runs along the edge in the opposite direction
#pragma unroll
            for (int a = 1; a < NX; a += 2) {
                txp[a] = -txp[a]; tUp[a] = -tUp[a]; tVp[a] = -tVp[a]; tup[a] = -tup[a]; tvp[a] = -tvp[a];
            }
#pragma unroll
            for (int a = 0; a < NX; ++a) {
                unp[a] = fma(tup[a], nx, tvp[a] * ny);
                qnp[a] = fma(tUp[a], nx, tVp[a] * ny);
            }
            xbp = Real(SQRT2) * x0;
            unbp = fabs(fma(Real(SQRT2) * u0, nx, Real(SQRT2) * v0 * ny));
        } else if (nb == NB_LAND) {
            // mirror: xi+ = xi-, normal parts of q and u change sign
            Real m2;
        if constexpr (std::is_same<Real, double>::value)
            m2 = -2.0 / len2;
        else
            m2 = -2.0f * rcp_approx(float(len2));
#pragma unroll
            for (int a = 0; a < NX; ++a) {
                txp[a] = txm[a];
                unp[a] = -unm[a];
                qnp[a] = -qnm[a];
                tUp[a] = fma(m2 * qnm[a], nx, tUm[a]);
                tVp[a] = fma(m2 * qnm[a], ny, tVm[a]);
            }
            xbp = xbm;
            unbp = unbm;
        } else {
            // open sea: xi+ = xi_hat(t), q and u copied
#pragma unroll
            for (int a = 0; a < NX; ++a) {
                txp[a] = a == 0 ? Real(xihat) : Real(0);
                tUp[a] = tUm[a];
                tVp[a] = tVm[a];
                unp[a] = unm[a];
                qnp[a] = qnm[a];
            }
            xbp = Real(xihat);
            unbp = unbm;
        }
        // penalty from constant parts at the edge midpoint (eq:lambda), times |E|
        Real lam;
        if constexpr (std::is_same<Real, double>::value)
            lam = tmax(unbm, unbp) + sqrt(g * (tmax(xbm, xbp) + hmid) * len2);
        else
            lam = tmax(unbm, unbp) + sqrt_approx(float(g * (double(tmax(xbm, xbp)) + hmid) * len2));
        // the flux's factor 1/2 rides on the scale (exact: a power of two)
        const Real sc = Real(0.5 * dt_det);
        const Real hg = Real(0.5 * g);
        Real FX[NT], FU[NT], FV[NT];
        double FW[NT];
        double xs[NX];
#pragma unroll
        for (int a = 0; a < NX; ++a) xs[a] = double(txm[a]) + double(txp[a]);
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const Real pb = hg * (prod1<NX, Real>(c, txm, txm) + prod1<NX, Real>(c, txp, txp));
            const Real mU = prod1<NX, Real>(c, tUm, unm) + prod1<NX, Real>(c, tUp, unp);
            const Real mV = prod1<NX, Real>(c, tVm, unm) + prod1<NX, Real>(c, tVp, unp);
            Real fx = qnm[c] + qnp[c] + lam * (txm[c] - txp[c]);
            if (nb == NB_LAND) fx = 0;   // q.n = 0: no mass flux through land
            FX[c] = sc * fx;
            FU[c] = sc * (mU + pb * nx + lam * (tUm[c] - tUp[c]));
            FV[c] = sc * (mV + pb * ny + lam * (tVm[c] - tVp[c]));
            // bathymetry part of the pressure, (P- + P+)/2 = g (xi- + xi+) h_b / 2
            double w = 0.0;
#pragma unroll
            for (int a = 0; a < NX; ++a)
#pragma unroll
                for (int b = 0; b < 2 && b < NX; ++b)
                    if (TG[c][a][b] != 0.0) w = fma(TG[c][a][b] * hbt[b], xs[a], w);
            FW[c] = 0.5 * g * w * dt_det;
        }
        double FWx[NT], FWy[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            FWx[c] = FW[c] * dy;
            FWy[c] = FW[c] * -dx;
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            Real a0 = A.L[0][q], a1 = A.L[1][q], a2 = A.L[2][q];
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                if (TR[k][q][c] == 0.0) continue;
                const Real r = Real(TR[k][q][c]);
                a0 = fma(-r, FX[c], a0);
                a1 = fma(-r, FU[c], a1);
                a2 = fma(-r, FV[c], a2);
            }
            A.L[0][q] = a0; A.L[1][q] = a1; A.L[2][q] = a2;
            double w0 = A.w(0, q), w1 = A.w(1, q);
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                if (TR[k][q][c] == 0.0) continue;
                w0 = fma(-TR[k][q][c], FWx[c], w0);
                w1 = fma(-TR[k][q][c], FWy[c], w1);
            }
            A.w(0, q) = w0; A.w(1, q) = w1;
        }
    }
}

template <int P, int PN, typename Real>
SWE_HD void edge_terms(const MeshView &m, unsigned e, const Buf<Real> &bC, const Buf<Real> &bU,
                                           const Buf<int> &bNb,
                                           const Fields<P, Real> &s, const Geo &G, double g,
                                           double xihat, double dt,
                                           const Real (*sR)[Ord<PN>::K][(P > PN ? P : PN) + 1],
                                           Acc<P, Real> &A)
{
    edge_one<P, PN, Real, 0>(m, e, bC, bU, bNb, s, G, g, xihat, dt, sR, A);
    edge_one<P, PN, Real, 1>(m, e, bC, bU, bNb, s, G, g, xihat, dt, sR, A);
    edge_one<P, PN, Real, 2>(m, e, bC, bU, bNb, s, G, g, xihat, dt, sR, A);
}

// ------------------------------------------------------------ u H = q
// H_ij = sum_{n < K(max(deg i, deg j))} xi_n C[n][i][j] + sum_{n<3} hb_n C[n][i][j];
// modes at or above Ke are masked to the identity (element order below P).
template <int P, typename Real>
SWE_HD void solve_u(const Real (&xi)[Ord<P>::K], const Real (&U)[Ord<P>::K],
                                        const Real (&V)[Ord<P>::K], const double (&hbh)[3], int Ke,
                                        Real (&u)[Ord<P>::K], Real (&v)[Ord<P>::K])
{
    constexpr int K = Ord<P>::K;
    constexpr bool dbl = std::is_same<Real, double>::value;
    // FP32: the total depth's modes H_n = xi_n + hb_n formed once (hb is
    // linear: modes 0-2), H is needed to FP32's relative accuracy only;
    // FP64: the bathymetry part summed on its own
    Real Hm[K];
#pragma unroll
    for (int n = 0; n < K; ++n) Hm[n] = (!dbl && n < 3) ? xi[n] + Real(hbh[n < 3 ? n : 0]) : xi[n];
    Real M[K][K];
#pragma unroll
    for (int i = 0; i < K; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            const int dmax = TDEG[i] > TDEG[j] ? TDEG[i] : TDEG[j];
            const int kt = KOFP[dmax];
            Real acc = 0;
#pragma unroll
            for (int n = 0; n < kt; ++n)
                if (TC[n][i][j] != 0.0) acc = fma(Real(TC[n][i][j]), Hm[n], acc);
            if constexpr (dbl) {
                double hbp = 0.0;
#pragma unroll
                for (int n = 0; n < 3; ++n)
                    if (TC[n][i][j] != 0.0) hbp = fma(TC[n][i][j], hbh[n], hbp);
                acc += Real(hbp);
            }
            if (i >= Ke || j >= Ke) acc = (i == j) ? Real(1) : Real(0);
            M[i][j] = acc;
        }
    // LDL^T without pivoting: H is symmetric positive definite for positive depth
    Real d[K], id[K];
#pragma unroll
    for (int j = 0; j < K; ++j) {
        Real djj = M[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) djj = fma(-M[j][k] * d[k], M[j][k], djj);
        d[j] = djj;
        if constexpr (std::is_same<Real, double>::value)
            id[j] = 1.0 / djj;
        else
            id[j] = rcp_approx(djj);
#pragma unroll
        for (int i = j + 1; i < K; ++i) {
            Real sij = M[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) sij = fma(-M[i][k] * d[k], M[j][k], sij);
            M[i][j] = sij * id[j];
        }
    }
    Real y[K], z[K];
#pragma unroll
    for (int i = 0; i < K; ++i) {
        Real a = i < Ke ? U[i] : Real(0), b = i < Ke ? V[i] : Real(0);
#pragma unroll
        for (int k = 0; k < i; ++k) {
            a = fma(-M[i][k], y[k], a);
            b = fma(-M[i][k], z[k], b);
        }
        y[i] = a;
        z[i] = b;
    }
#pragma unroll
    for (int i = 0; i < K; ++i) { y[i] *= id[i]; z[i] *= id[i]; }
#pragma unroll
    for (int i = K - 1; i >= 0; --i) {
        Real a = y[i], b = z[i];
#pragma unroll
        for (int k = i + 1; k < K; ++k) {
            a = fma(-M[k][i], u[k], a);
            b = fma(-M[k][i], v[k], b);
        }
        u[i] = a;
        v[i] = b;
    }
}

SWE_HD void hb_modes(const Geo &G, double (&hbh)[3])
{
#pragma unroll
    for (int n = 0; n < 3; ++n) hbh[n] = TW[n][0] * G.h[0] + TW[n][1] * G.h[1] + TW[n][2] * G.h[2];
}

// ------------------------------------------------------------ kernel pieces
template <int KN, int NX, typename Real>
__device__ __forceinline__ void load_trace_table(Real (*sR)[KN][NX])
{
    for (int i = threadIdx.x; i < 3 * KN * NX; i += blockDim.x) {
        const int k = i / (KN * NX), r = i % (KN * NX);
        sR[k][r / NX][r % NX] = (r % NX) < 4 ? Real(TR[k][r / NX][r % NX]) : Real(0);
    }
}

template <int P, typename Real>
SWE_HD void acc_init(Acc<P, Real> &A, const Fields<P, Real> &s, bool with_state)
{
#pragma unroll
    for (int q = 0; q < Ord<P>::K; ++q) {
        A.L[0][q] = with_state ? s.xi[q] : Real(0);
        A.L[1][q] = with_state ? s.U[q] : Real(0);
        A.L[2][q] = with_state ? s.V[q] : Real(0);
        if constexpr (Acc<P, Real>::SPLIT) { A.W[0][q] = 0.0; A.W[1][q] = 0.0; }
    }
}

// acc += dt L(c) for one element of order P with neighbours of order <= PN
template <int P, int PN, typename Real>
SWE_HD void element_rhs(const StageArgs<Real> &a, unsigned e, const Buf<Real> &bC,
                                            const Buf<Real> &bU, const Buf<int> &bNb,
                                            const Fields<P, Real> &s, const Geo &G, const double (&hbh)[3],
                                            double dt, const Real (*sR)[Ord<PN>::K][(P > PN ? P : PN) + 1],
                                            Acc<P, Real> &A, double xihat)
{
    constexpr int K = Ord<P>::K;
    volume_term<P, Real>(s, hbh, G, a.ph.g, dt, A);
    source_term<P, Real>(s, G, a.ph, dt, A);
    edge_terms<P, PN, Real>(a.m, e, bC, bU, bNb, s, G, a.ph.g, xihat, dt, sR, A);
    if constexpr (Acc<P, Real>::SPLIT) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            A.L[1][q] += Real(A.W[0][q]);
            A.L[2][q] += Real(A.W[1][q]);
        }
    }
    if (a.src) {
        const Buf<Real> bS(a.src, 3 * a.m.KS, a.m.stride);
        const Real rdt = Real(dt);
        const unsigned off = e * (unsigned)sizeof(Real);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int q = 0; q < K; ++q) A.L[j][q] = fma(rdt, bS.ld(j * a.m.KS + q, off), A.L[j][q]);
    }
}

// SSP-RK2 combine of acc = c + dt L, u-solve of the new state, store, depth check
template <int P, typename Real, int MODE>
__device__ __forceinline__ void finish_stage(const StageArgs<Real> &a, unsigned e, const Geo &G,
                                             const double (&hbh)[3], int Ke, const Real (&L)[3][Ord<P>::K],
                                             int *flag)
{
    constexpr int K = Ord<P>::K;
    const int KS = a.m.KS, stride = a.m.stride;
    const unsigned off = e * (unsigned)sizeof(Real);
    Real xn[K], Un[K], Vn[K];
    const Buf<Real> bN(a.Cn, 3 * KS, stride);
#pragma unroll
    for (int q = 0; q < K; ++q) {
        Real c0 = L[0][q], c1 = L[1][q], c2 = L[2][q];
        if constexpr (MODE == MODE_STAGE2) {
            c0 = Real(0.5) * bN.ld(0 * KS + q, off) + Real(0.5) * c0;
            c1 = Real(0.5) * bN.ld(1 * KS + q, off) + Real(0.5) * c1;
            c2 = Real(0.5) * bN.ld(2 * KS + q, off) + Real(0.5) * c2;
        }
        xn[q] = c0; Un[q] = c1; Vn[q] = c2;
    }
    Real un[K], vn[K];
    solve_u<P, Real>(xn, Un, Vn, hbh, Ke, un, vn);
    Real chk = 0;
    const Buf<Real> bO(a.Cout, 3 * KS, stride), bV(a.Uout, 2 * KS, stride);
    // FP64 results are streamed past the caches (measured: 4 % shorter FP64
    // stages at p = 2, while the same policy lengthens FP32 stages by 4 %)
    constexpr bool stream = sizeof(Real) == 8;
#pragma unroll
    for (int q = 0; q < K; ++q) {
        if constexpr (stream) {
            bO.st_stream(0 * KS + q, off, xn[q]);
            bO.st_stream(1 * KS + q, off, Un[q]);
            bO.st_stream(2 * KS + q, off, Vn[q]);
            bV.st_stream(0 * KS + q, off, un[q]);
            bV.st_stream(1 * KS + q, off, vn[q]);
        } else {
            bO.st(0 * KS + q, off, xn[q]);
            bO.st(1 * KS + q, off, Un[q]);
            bO.st(2 * KS + q, off, Vn[q]);
            bV.st(0 * KS + q, off, un[q]);
            bV.st(1 * KS + q, off, vn[q]);
        }
        chk += xn[q] + Un[q] + Vn[q] + un[q] + vn[q];
    }
    const double Hmean = SQRT2 * double(xn[0]) + (G.h[0] + G.h[1] + G.h[2]) * (1.0 / 3.0);
    if (!(Hmean > 0.0) || !isfinite(chk)) flag[0] = 1;
}

// ------------------------------------------------------------ shared edge fluxes
// Stage kernel in which each edge flux inside a block of BLOCK consecutive
// elements is computed once and handed to both sides through LDS (the passes
// are described at stage_sh_block).  The block's edge items are host-built:
// a pair of elements of the block (taken once, from the lower index), an
// element and a neighbour outside the block, a land or an open edge.  An
// item packs a (bits 0-7), its local edge (8-9), b (10-17), b's local edge
// (18-19) and the kind (20-21).
constexpr unsigned EK_PAIR = 0, EK_EXT = 1, EK_LAND = 2, EK_OPEN = 3;

// Waves per SIMD the shared-flux kernels are built for at least: what their
// LDS allows and their registers reach without spilling (FP32 p = 2: 32 KB
// per 256-element block, four blocks per CU, 128 registers; FP32 p = 1:
// 22 KB, five waves at 85 registers; FP32 p = 3 and FP64 p = 2: 53 and 63 KB,
// two waves (three would spill); FP64 p = 1: 34 KB, three waves (four would
// spill); FP64 p = 3: 105 KB, one block, whose registers then spill into
// accumulation registers rather than scratch).
template <int P, typename Real>
constexpr int sh_waves()
{
    constexpr bool dbl = std::is_same<Real, double>::value;
    return dbl ? (P == 1 ? 3 : P == 3 ? 1 : 2) : (P == 2 ? 4 : P == 3 ? 2 : 3);
}

// The batch form at FP32 order 3 loads the geometry after the edge pass and
// runs three waves per SIMD (168 registers, no spill; its LDS, 53 KB per
// block, allows three blocks per CU); the single-instance form, which also
// carries the separated scheme's base-pass paths, would spill there.
template <int P, typename Real>
constexpr bool batch_sh_fp32p3()
{
    return !std::is_same<Real, double>::value && P == 3;
}

// Per-block LDS.  The state copy C is read by the edge pass only; the
// per-item results F, W are written after it (every lane holds its items'
// results in registers across a barrier), so the two share the storage.
// Results are stored per edge item (lane i writes column i: consecutive
// words, no bank conflicts), and slot[k][l] tells element l which item
// holds its local edge k (bit 15: l is the item's second side, which sees
// the flux negated and reversed along the edge).
template <int P, typename Real>
struct ShLds {
    static constexpr int K = Ord<P>::K, NT = Ord<P>::NT;
    Real R[3][K][NT];              // trace matrices
    unsigned short slot[3][BLOCK]; // item of each (local edge, element)
    union {
        Real C[5 * K][BLOCK];      // xi, U, V, u, v modes of the block's elements
        struct {
            Real F[3 * NT][2 * BLOCK];  // flux modes (component, mode) per item
            double W[NT][2 * BLOCK];    // bathymetry part of the pressure flux, FP64, per item
        } E;
    } U;
};

// An edge item's results, kept in registers until the state copy is no
// longer read.
template <int P, typename Real>
struct ShItem {
    static constexpr int NT = Ord<P>::NT;
    Real F[3][NT];
    double W[NT];
};

template <int P, typename Real>
__device__ __forceinline__ void traces_of(const ShLds<P, Real> &S, int l, int k, Real (&t)[5][Ord<P>::NT])
{
    constexpr int K = Ord<P>::K, NT = Ord<P>::NT;
#pragma unroll
    for (int f = 0; f < 5; ++f)
#pragma unroll
        for (int c = 0; c < NT; ++c) t[f][c] = Real(0);
#pragma unroll
    for (int n = 0; n < K; ++n)
#pragma unroll
        for (int c = 0; c < NT && c <= TDEG[n]; ++c) {
            const Real r = S.R[k][n][c];
#pragma unroll
            for (int f = 0; f < 5; ++f) t[f][c] = fma(S.U.C[f * K + n][l], r, t[f][c]);
        }
}

template <int P, typename Real>
__device__ __forceinline__ void load_trace_lds(ShLds<P, Real> &S)
{
    constexpr int K = Ord<P>::K, NT = Ord<P>::NT;
    for (int i = threadIdx.x; i < 3 * K * NT; i += BLOCK) {
        const int k = i / (K * NT), r = i % (K * NT);
        S.R[k][r / NT][r % NT] = Real(TR[k][r / NT][r % NT]);
    }
}

// The Lax-Friedrichs flux of one edge item, in the first side's orientation,
// times two (its factor 1/2 is applied with dt / |det B| at the lift) and
// unscaled by dt / |det B| (the edge pass of the shared-flux kernels); the
// FP64 bathymetry part W is complete.
template <int P, typename Real>
__device__ __forceinline__ void sh_flux(const ShLds<P, Real> &S, const MeshView &m, const Buf<Real> &bC,
                                        const Buf<Real> &bU, const Buf<int> &bEv, const Buf<int> &bNb, unsigned e0,
                                        unsigned w, double xihat, double g, ShItem<P, Real> &out)
{
    constexpr int K = Ord<P>::K, NT = Ord<P>::NT;
    const int KS = m.KS;
    const int la = (int)(w & 255u), ka = (int)((w >> 8) & 3u), lb = (int)((w >> 10) & 255u);
    const int kb = (int)((w >> 18) & 3u);
    const unsigned kind = (w >> 20) & 3u;
    const unsigned ea = e0 + (unsigned)la;
    const int va = (ka + 1) % 3, vb = (ka + 2) % 3;
    const double4 pa = m.vtx[(unsigned)bEv.ld(va, ea * 4u)];
    const double4 pb = m.vtx[(unsigned)bEv.ld(vb, ea * 4u)];
    const double dx = pb.x - pa.x, dy = pb.y - pa.y;
    const double len2 = dx * dx + dy * dy;
    const Real nx = Real(dy), ny = Real(-dx);          // |E| n of side a
    const double hmid = 0.5 * (pa.z + pb.z);
    const double hbt[2] = {hmid, (pb.z - pa.z) * INV_2SQRT3};
    Real tm[5][NT], tp[5][NT];
    traces_of<P, Real>(S, la, ka, tm);
    const Real xbm = Real(SQRT2) * S.U.C[0][la];
    const Real unbm = fabs(fma(Real(SQRT2) * S.U.C[3 * K][la], nx, Real(SQRT2) * S.U.C[4 * K][la] * ny));
    Real unm[NT], qnm[NT], unp[NT], qnp[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        unm[c] = fma(tm[3][c], nx, tm[4][c] * ny);
        qnm[c] = fma(tm[1][c], nx, tm[2][c] * ny);
    }
    Real xbp, unbp;
    if (kind == EK_PAIR || kind == EK_EXT) {
        Real x0, u0, v0;
        if (kind == EK_PAIR) {
            traces_of<P, Real>(S, lb, kb, tp);
            x0 = S.U.C[0][lb];
            u0 = S.U.C[3 * K][lb];
            v0 = S.U.C[4 * K][lb];
        } else {
            const int nb = bNb.ld(ka, ea * 4u);
            const int kk = (m.enbk[ea] >> (2 * ka)) & 3;
            const unsigned un_ = (unsigned)nb * (unsigned)sizeof(Real);
#pragma unroll
            for (int f = 0; f < 5; ++f)
#pragma unroll
                for (int c = 0; c < NT; ++c) tp[f][c] = Real(0);
            x0 = Real(0); u0 = Real(0); v0 = Real(0);
#pragma unroll
            for (int n = 0; n < K; ++n) {
                const Real fv[5] = {bC.ld(0 * KS + n, un_), bC.ld(1 * KS + n, un_), bC.ld(2 * KS + n, un_),
                                    bU.ld(0 * KS + n, un_), bU.ld(1 * KS + n, un_)};
                if (n == 0) { x0 = fv[0]; u0 = fv[3]; v0 = fv[4]; }
#pragma unroll
                for (int c = 0; c < NT && c <= TDEG[n]; ++c) {
                    const Real r = S.R[kk][n][c];
#pragma unroll
                    for (int f = 0; f < 5; ++f) tp[f][c] = fma(fv[f], r, tp[f][c]);
                }
            }
        }
        // the other side runs along the edge in the opposite direction
#pragma unroll
        for (int c = 1; c < NT; c += 2)
#pragma unroll
            for (int f = 0; f < 5; ++f) tp[f][c] = -tp[f][c];
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            unp[c] = fma(tp[3][c], nx, tp[4][c] * ny);
            qnp[c] = fma(tp[1][c], nx, tp[2][c] * ny);
        }
        xbp = Real(SQRT2) * x0;
        unbp = fabs(fma(Real(SQRT2) * u0, nx, Real(SQRT2) * v0 * ny));
    } else if (kind == EK_LAND) {
        // mirror: xi+ = xi-, normal parts of q and u change sign
        Real m2;
        if constexpr (std::is_same<Real, double>::value)
            m2 = -2.0 / len2;
        else
            m2 = -2.0f * rcp_approx(float(len2));
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            tp[0][c] = tm[0][c];
            unp[c] = -unm[c];
            qnp[c] = -qnm[c];
            tp[1][c] = fma(m2 * qnm[c], nx, tm[1][c]);
            tp[2][c] = fma(m2 * qnm[c], ny, tm[2][c]);
        }
        xbp = xbm;
        unbp = unbm;
    } else {
        // open sea: xi+ = xi_hat(t), q and u copied
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            tp[0][c] = c == 0 ? Real(xihat) : Real(0);
            tp[1][c] = tm[1][c];
            tp[2][c] = tm[2][c];
            unp[c] = unm[c];
            qnp[c] = qnm[c];
        }
        xbp = Real(xihat);
        unbp = unbm;
    }
    // penalty from constant parts at the edge midpoint (eq:lambda), times |E|
    Real lam;
    if constexpr (std::is_same<Real, double>::value)
        lam = tmax(unbm, unbp) + sqrt(g * (tmax(xbm, xbp) + hmid) * len2);
    else
        lam = tmax(unbm, unbp) + sqrt_approx(float(g * (double(tmax(xbm, xbp)) + hmid) * len2));
    const Real hg = Real(0.5 * g);
    Real (&F)[3][NT] = out.F;
    double (&Wf)[NT] = out.W;
#pragma unroll
    for (int c = 0; c < NT; ++c) {
        const Real pb = hg * (prod1<NT, Real>(c, tm[0], tm[0]) + prod1<NT, Real>(c, tp[0], tp[0]));
        const Real mU = prod1<NT, Real>(c, tm[1], unm) + prod1<NT, Real>(c, tp[1], unp);
        const Real mV = prod1<NT, Real>(c, tm[2], unm) + prod1<NT, Real>(c, tp[2], unp);
        Real fx = qnm[c] + qnp[c] + lam * (tm[0][c] - tp[0][c]);
        if (kind == EK_LAND) fx = 0;   // q.n = 0: no mass flux through land
        F[0][c] = fx;
        F[1][c] = mU + pb * nx + lam * (tm[1][c] - tp[1][c]);
        F[2][c] = mV + pb * ny + lam * (tm[2][c] - tp[2][c]);
        // bathymetry part of the pressure, (P- + P+)/2 = g (xi- + xi+) h_b / 2
        double wv = 0.0;
#pragma unroll
        for (int aa = 0; aa < NT; ++aa) {
            const double xs = double(tm[0][aa]) + double(tp[0][aa]);
#pragma unroll
            for (int bb = 0; bb < 2 && bb < NT; ++bb)
                if (TG[c][aa][bb] != 0.0) wv = fma(TG[c][aa][bb] * hbt[bb], xs, wv);
        }
        Wf[c] = 0.5 * g * wv;
    }
}

// Store item i's flux in its column and point its sides' slots at it (the
// second side of a pair inside the block marked by bit 15).
template <int P, typename Real>
__device__ __forceinline__ void sh_store(ShLds<P, Real> &S, int i, unsigned w, const ShItem<P, Real> &r)
{
    constexpr int NT = Ord<P>::NT;
    const int la = (int)(w & 255u), ka = (int)((w >> 8) & 3u), lb = (int)((w >> 10) & 255u);
    const int kb = (int)((w >> 18) & 3u);
#pragma unroll
    for (int c = 0; c < NT; ++c) {
#pragma unroll
        for (int j = 0; j < 3; ++j) S.U.E.F[j * NT + c][i] = r.F[j][c];
        S.U.E.W[c][i] = r.W[c];
    }
    S.slot[ka][la] = (unsigned short)i;
    if (((w >> 20) & 3u) == EK_PAIR) S.slot[kb][lb] = (unsigned short)(i | 0x8000);
}

// The passes over the block of elements [e0, e0 + BLOCK) (live below e_end),
// whose edge items are items[0, nitems), nitems <= 2 BLOCK (ITEM_PAD slots
// among them are empty).  Every thread of
// the block calls it (it holds three block barriers); the trace tables in S
// are loaded before (the first barrier orders them before their first use).
//   1. each lane (one element) loads its state into registers and copies it
//      to LDS;
//   2. each lane computes the flux of at most two edge items (a pair of
//      elements of the block, an element and a neighbour outside it, a land
//      or an open edge) from the state copies and keeps it in registers;
//      once every lane is done reading the copies, the fluxes overwrite them,
//      each stored for its first side and, for a pair, for the second;
//   3. each lane adds its volume and source terms, lifts its three edge
//      fluxes with its own geometry and finishes the stage.
template <int P, typename Real, int MODE, bool EARLY_GEO = !std::is_same<Real, double>::value && P == 3>
__device__ __forceinline__ void stage_sh_block(ShLds<P, Real> &S, const StageArgs<Real> &a, unsigned e0,
                                               unsigned e_end, const unsigned *items, int nitems, double xihat,
                                               double dt, int *flag)
{
    constexpr int K = Ord<P>::K, NT = Ord<P>::NT;
    const MeshView &m = a.m;
    const int KS = m.KS, stride = m.stride;
    const unsigned l = threadIdx.x, e = e0 + l;
    const bool live = e < e_end;
    if (MODE == MODE_RHS) dt = 1.0;
    const Buf<Real> bC(a.Cin, 3 * KS, stride), bU(a.Uin, 2 * KS, stride);
    const Buf<int> bEv(m.ev, 3, stride), bNb(m.enb, 3, stride);
    const double g = a.ph.g;

    // 1. state to registers and LDS; at FP32 order 3 (two waves per SIMD) also
    //    the geometry, whose latency then hides behind the edge pass (elsewhere
    //    the registers it would hold across that pass cost a wave per SIMD:
    //    only the vertex ids are loaded here, the vertices after the edge pass)
    constexpr bool early_geo = EARLY_GEO;
    Fields<P, Real> s;
    Geo G;
    double hbh[3];
    int id3[3] = {0, 0, 0};
    const unsigned off = e * (unsigned)sizeof(Real);
    if (live) {
        if constexpr (early_geo) {
            load_geo(m.vtx, bEv, e * 4u, G);
        } else {
#pragma unroll
            for (int v = 0; v < 3; ++v) id3[v] = bEv.ld(v, e * 4u);
        }
        load_state<P, Real>(bC, bU, KS, off, s);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            S.U.C[0 * K + q][l] = s.xi[q];
            S.U.C[1 * K + q][l] = s.U[q];
            S.U.C[2 * K + q][l] = s.V[q];
            S.U.C[3 * K + q][l] = s.u[q];
            S.U.C[4 * K + q][l] = s.v[q];
        }
    }
    __syncthreads();

    // 2. the fluxes of this lane's (at most two) edge items
    const int n = nitems < 2 * BLOCK ? nitems : 2 * BLOCK;
    const int it0 = (int)l, it1 = (int)l + BLOCK;
    const unsigned w0 = it0 < n ? items[it0] : ITEM_PAD, w1 = it1 < n ? items[it1] : ITEM_PAD;
    ShItem<P, Real> r0, r1;
    if (w0 != ITEM_PAD) sh_flux<P, Real>(S, m, bC, bU, bEv, bNb, e0, w0, xihat, g, r0);
    if (w1 != ITEM_PAD) sh_flux<P, Real>(S, m, bC, bU, bEv, bNb, e0, w1, xihat, g, r1);
    __syncthreads();
    if (w0 != ITEM_PAD) sh_store<P, Real>(S, it0, w0, r0);
    if (w1 != ITEM_PAD) sh_store<P, Real>(S, it1, w1, r1);
    __syncthreads();
    if (!live) return;
    // base pass of the order-partitioned scheme: a listed element belongs to
    // the full-order kernel of its order (the fluxes of its edges above were
    // taken at the base order, which is exact only for unlisted elements,
    // whose neighbours all have the base order)
    const bool listed = a.inlist && a.inlist[e];
    if (a.skip_listed && listed) return;

    // 3. volume and source terms, the three edge fluxes lifted, the stage finished
    if constexpr (!early_geo) geo_from_ids(m.vtx, id3, G);
    hb_modes(G, hbh);
    Acc<P, Real> A;
    acc_init<P, Real>(A, s, MODE != MODE_RHS);
    volume_term<P, Real>(s, hbh, G, g, dt, A);
    source_term<P, Real>(s, G, a.ph, dt, A);
    const double dt_det = dt * G.idet;
    // the stored fluxes lack their factor 1/2: the scale carries it (exact)
    const Real sc = Real(0.5 * dt_det);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int ka = (k + 1) % 3, kb = (k + 2) % 3;
        const double dx = G.X[kb] - G.X[ka], dy = G.Y[kb] - G.Y[ka];
        // the item of this edge; as its second side the flux comes negated and
        // reversed along the edge (even Legendre modes change sign, odd ones not)
        const unsigned sl = S.slot[k][l];
        const int it = (int)(sl & 0x7fffu);
        const bool second = (sl & 0x8000u) != 0u;
        Real FX[NT], FU[NT], FV[NT];
        double FWx[NT], FWy[NT];
#pragma unroll
        for (int c = 0; c < NT; ++c) {
            const bool flip = second && !(c & 1);
            const Real f0 = S.U.E.F[0 * NT + c][it], f1 = S.U.E.F[1 * NT + c][it], f2 = S.U.E.F[2 * NT + c][it];
            FX[c] = sc * (flip ? -f0 : f0);
            FU[c] = sc * (flip ? -f1 : f1);
            FV[c] = sc * (flip ? -f2 : f2);
            const double w = S.U.E.W[c][it];
            const double FW = (second && (c & 1) ? -w : w) * dt_det;
            FWx[c] = FW * dy;
            FWy[c] = FW * -dx;
        }
#pragma unroll
        for (int q = 0; q < K; ++q) {
            Real a0 = A.L[0][q], a1 = A.L[1][q], a2 = A.L[2][q];
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                if (TR[k][q][c] == 0.0) continue;
                const Real r = Real(TR[k][q][c]);
                a0 = fma(-r, FX[c], a0);
                a1 = fma(-r, FU[c], a1);
                a2 = fma(-r, FV[c], a2);
            }
            A.L[0][q] = a0; A.L[1][q] = a1; A.L[2][q] = a2;
            double w0 = A.w(0, q), w1 = A.w(1, q);
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                if (TR[k][q][c] == 0.0) continue;
                w0 = fma(-TR[k][q][c], FWx[c], w0);
                w1 = fma(-TR[k][q][c], FWy[c], w1);
            }
            A.w(0, q) = w0; A.w(1, q) = w1;
        }
    }
    if constexpr (Acc<P, Real>::SPLIT) {
#pragma unroll
        for (int q = 0; q < K; ++q) {
            A.L[1][q] += Real(A.W[0][q]);
            A.L[2][q] += Real(A.W[1][q]);
        }
    }
    if (a.src) {
        const Buf<Real> bS(a.src, 3 * KS, stride);
        const Real rdt = Real(dt);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int q = 0; q < K; ++q) A.L[j][q] = fma(rdt, bS.ld(j * KS + q, off), A.L[j][q]);
    }
    if constexpr (MODE == MODE_RHS) {
        const Buf<Real> bL(a.Lout, 3 * KS, stride);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int q = 0; q < K; ++q) bL.st(j * KS + q, off, A.L[j][q]);
    } else {
        if (a.Lb && listed) {
            // base pass of the order-separated scheme: the listed element's
            // base part waits in Lb for the epilogue
            const Buf<Real> bB(a.Lb, 3 * K, stride);
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int q = 0; q < K; ++q) bB.st(j * K + q, off, A.L[j][q]);
            return;
        }
        finish_stage<P, Real, MODE>(a, e, G, hbh, K, A.L, flag);
    }
}

template <int P, typename Real, int MODE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(sh_waves<P, Real>(), 8)))
k_stage_sh(StageArgs<Real> a, const unsigned *items, const int *item_off)
{
    __shared__ ShLds<P, Real> S;
    load_trace_lds<P, Real>(S);
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    double xihat = a.xihat, dt = a.dt;
    if (a.inst) {
        // the step's clock stopped (failure): the whole block leaves before its first barrier
        if (!a.inst->run) return;
        xihat = MODE == MODE_STAGE2 ? a.inst->xh[1] : a.inst->xh[0];
        dt = a.inst->dt;
    }
    const int i0 = item_off[blk], i1 = item_off[blk + 1];
    stage_sh_block<P, Real, MODE>(S, a, (unsigned)blk * BLOCK, (unsigned)a.m.ne, items + i0, i1 - i0, xihat, dt,
                                  a.flag);
}

// ------------------------------------------------------------ kernels
// Full stage of every element at one order P (unseparated scheme), or, with
// SEP, the base part of the order-separated scheme: every element evaluated
// with its first K(P) modes (P = p_base); elements whose right-hand side also
// has a correction store their partial stage value in Lb for the epilogue.
template <int P, typename Real, int MODE, bool SEP>
__device__ __forceinline__ void stage_element(const StageArgs<Real> &a, unsigned e,
                                              const Real (*sR)[Ord<P>::K][Ord<P>::NT], double xihat,
                                              double dt_stage, int *flag)
{
    constexpr int K = Ord<P>::K;
    if constexpr (SEP) {
        if (a.skip_listed && a.inlist[e]) return;   // a full-order kernel owns this element
    }
    const MeshView &m = a.m;
    const int KS = m.KS, stride = m.stride;
    const unsigned off = e * (unsigned)sizeof(Real);
    const Buf<Real> bC(a.Cin, 3 * KS, stride), bU(a.Uin, 2 * KS, stride);
    const Buf<int> bEv(m.ev, 3, stride), bNb(m.enb, 3, stride);
    Geo G;
    load_geo(m.vtx, bEv, e * 4u, G);
    double hbh[3];
    hb_modes(G, hbh);
    Fields<P, Real> s;
    load_state<P, Real>(bC, bU, KS, off, s);
    const int Ke = (!SEP && a.mixed) ? KOFP[m.ep[e]] : K;

    const double dt = MODE == MODE_RHS ? 1.0 : dt_stage;
    Acc<P, Real> A;
    acc_init<P, Real>(A, s, MODE != MODE_RHS);
    element_rhs<P, P, Real>(a, e, bC, bU, bNb, s, G, hbh, dt, sR, A, xihat);
    if (!SEP && a.mixed) {
        // modes above the element's order stay zero
#pragma unroll
        for (int q = 0; q < K; ++q)
            if (q >= Ke) { A.L[0][q] = 0; A.L[1][q] = 0; A.L[2][q] = 0; }
    }
    if constexpr (MODE == MODE_RHS) {
        const Buf<Real> bL(a.Lout, 3 * KS, stride);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int q = 0; q < K; ++q) bL.st(j * KS + q, off, A.L[j][q]);
        return;
    } else {
        if constexpr (SEP) {
            if (a.inlist[e]) {
                const Buf<Real> bB(a.Lb, 3 * K, stride);
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int q = 0; q < K; ++q) bB.st(j * K + q, off, A.L[j][q]);
                return;
            }
        }
        finish_stage<P, Real, MODE>(a, e, G, hbh, Ke, A.L, flag);
    }
}

template <int P, typename Real, int MODE, bool SEP>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(waves_target<P, Real>(), 8)))
k_stage(StageArgs<Real> a)
{
    constexpr int K = Ord<P>::K, NT = Ord<P>::NT;
    __shared__ Real sR[3][K][NT];
    load_trace_table<K, NT, Real>(sR);
    __syncthreads();
    const unsigned le = (unsigned)xcd_block(blockIdx.x, gridDim.x) * BLOCK + threadIdx.x;
    if (le >= (unsigned)a.m.ne) return;
    double xihat = a.xihat, dt = a.dt;
    if (a.inst) {
        // one instance of a batch: its clock lives on the device
        if (!a.inst->run) return;
        xihat = MODE == MODE_STAGE2 ? a.inst->xh[1] : a.inst->xh[0];
        dt = a.inst->dt;
    }
    stage_element<P, Real, MODE, SEP>(a, le + (unsigned)a.e_off, sR, xihat, dt, a.flag);
}

// ------------------------------------------------------------ batched instances
// One launch per order class and stage covers the tiles of every resident
// instance of that order (one tile per block, no loop around the element
// evaluation).  All instances of an order share pooled arrays passed as
// kernel arguments; a tile (TILE consecutive elements of one instance) only
// reads its instance's scalars (step, open-sea elevation, physics, clock).
// Each XCD takes a contiguous eighth of the tile list, so the neighbour
// gathers of an instance's elements stay in one L2.  Instances whose clock
// says they are done are skipped: one step graph serves any resident set.
template <int P, typename Real, int MODE, int TILE>
__global__ void __launch_bounds__(TILE) __attribute__((amdgpu_waves_per_eu(waves_target<P, Real>(), 8)))
k_batch_stage(BatchArgs b)
{
    constexpr int K = Ord<P>::K, NT = Ord<P>::NT;
    __shared__ Real sR[3][K][NT];
    load_trace_table<K, NT, Real>(sR);
    __syncthreads();
    // One tile per block.  XCD x (blocks x, x+8, ...) owns the contiguous
    // eighth [lo, hi) of the tile list; the grid is sized from the tile
    // capacity (at least 8 blocks more than there can be tiles), so every
    // XCD has a block for each of its tiles and the surplus blocks exit.
    const int ntiles = b.ntiles[0];
    const int x = (int)(blockIdx.x & 7u), i = (int)(blockIdx.x >> 3);
    const int lo = (int)(((long long)ntiles * x) >> 3), hi = (int)(((long long)ntiles * (x + 1)) >> 3);
    const int t = lo + i;
    if (t >= hi) return;
    StageArgs<Real> a{};   // every field not set below is zero / null (no lists, no skipping)
    a.m.ne = 0;
    a.m.stride = b.pool.cap;
    a.m.KS = K;
    a.m.vtx = b.vtx;
    a.m.ev = b.pool.ev;
    a.m.enb = b.pool.nb;
    a.m.enbk = b.pool.nbk;
    a.m.ep = nullptr;
    a.Cin = static_cast<const Real *>(MODE == MODE_STAGE1 ? b.pool.C0 : b.pool.C1);
    a.Uin = static_cast<const Real *>(MODE == MODE_STAGE1 ? b.pool.U0 : b.pool.U1);
    a.Cn = static_cast<const Real *>(b.pool.C0);
    a.Cout = static_cast<Real *>(MODE == MODE_STAGE1 ? b.pool.C1 : b.pool.C0);
    a.Uout = static_cast<Real *>(MODE == MODE_STAGE1 ? b.pool.U1 : b.pool.U0);
    a.Lout = nullptr;
    a.src = nullptr;
    const int2 tile = b.tiles[t];
    const InstDesc &I = b.inst[tile.x];
    if (!I.run) return;
    // a member with per-element orders (a static order map or indicator-driven
    // orders) masks each element's modes by its order, as on its own
    a.m.ep = b.pool.ep;
    a.mixed = I.mixed;
    a.ph = I.ph;
    const unsigned e = (unsigned)tile.y + threadIdx.x;
    if (e < (unsigned)(I.first + I.ne))
        stage_element<P, Real, MODE, false>(a, e, sR, MODE == MODE_STAGE1 ? I.xh[0] : I.xh[1], I.dt,
                                            b.flags + tile.x);
}

// Shared-flux stage over the 256-element tiles of every resident instance of
// one order (one tile per block, tile list split by XCD as above).  A tile
// starts on a multiple of 256 within its instance, so the instance's edge
// items of that block (local indices) serve it unchanged.
template <int P, typename Real, int MODE>
__global__ void __launch_bounds__(BLOCK)
__attribute__((amdgpu_waves_per_eu(batch_sh_fp32p3<P, Real>() ? 3 : sh_waves<P, Real>(), 8)))
k_batch_stage_sh(BatchArgs b)
{
    __shared__ ShLds<P, Real> S;
    load_trace_lds<P, Real>(S);
    // the returns below are uniform over the block (tile and instance)
    const int ntiles = b.ntiles[0];
    const int x = (int)(blockIdx.x & 7u), i = (int)(blockIdx.x >> 3);
    const int lo = (int)(((long long)ntiles * x) >> 3), hi = (int)(((long long)ntiles * (x + 1)) >> 3);
    const int t = lo + i;
    if (t >= hi) return;
    const int2 tile = b.tiles[t];
    const InstDesc &I = b.inst[tile.x];
    if (!I.run) return;
    StageArgs<Real> a{};   // every field not set below is zero / null (no lists, no skipping)
    a.m.ne = 0;
    a.m.stride = b.pool.cap;
    a.m.KS = Ord<P>::K;
    a.m.vtx = b.vtx;
    a.m.ev = b.pool.ev;
    a.m.enb = b.pool.nb;
    a.m.enbk = b.pool.nbk;
    a.m.ep = nullptr;
    a.Cin = static_cast<const Real *>(MODE == MODE_STAGE1 ? b.pool.C0 : b.pool.C1);
    a.Uin = static_cast<const Real *>(MODE == MODE_STAGE1 ? b.pool.U0 : b.pool.U1);
    a.Cn = static_cast<const Real *>(b.pool.C0);
    a.Cout = static_cast<Real *>(MODE == MODE_STAGE1 ? b.pool.C1 : b.pool.C0);
    a.Uout = static_cast<Real *>(MODE == MODE_STAGE1 ? b.pool.U1 : b.pool.U0);
    a.Lout = nullptr;
    a.src = nullptr;
    a.mixed = 0;
    a.ph = I.ph;
    const unsigned e0 = (unsigned)tile.y;
    // the batch form loads the geometry after the edge pass at every order
    stage_sh_block<P, Real, MODE, false>(S, a, e0, (unsigned)(I.first + I.ne), b.pool.items + 3u * e0,
                                         b.pool.nitems[e0 / BLOCK], MODE == MODE_STAGE1 ? I.xh[0] : I.xh[1], I.dt,
                                         b.flags + tile.x);
}

// Copy an instance's edge items (blocks of 256 elements, item_off[nblk + 1])
// into the pool slots of its element range starting at first (a multiple
// of 256): one block per 256-element block.
__global__ void __launch_bounds__(BLOCK) k_place_items(const unsigned *items, const int *item_off, PoolView pool,
                                                       int first)
{
    const int j = blockIdx.x;
    const int i0 = item_off[j], n = item_off[j + 1] - i0;
    const int f = first + j * BLOCK;
    for (int k = threadIdx.x; k < n; k += BLOCK) pool.items[3 * f + k] = items[i0 + k];
    if (threadIdx.x == 0) pool.nitems[f / BLOCK] = n;
}

__global__ void __launch_bounds__(BLOCK) k_relocate(const int *ev, const int *nb, const unsigned char *nbk,
                                                    const signed char *ep, int ne, int stride, PoolView pool,
                                                    int first, int vbase)
{
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= ne) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        pool.ev[k * pool.cap + first + e] = ev[k * stride + e] + vbase;
        const int n = nb[k * stride + e];
        pool.nb[k * pool.cap + first + e] = n >= 0 ? n + first : n;
    }
    pool.nbk[first + e] = nbk[e];
    pool.ep[first + e] = ep[e];
}

// Per-step clock of every resident instance: open-sea elevation at the two
// stage times, then advance its time and step budget.
// Open-sea elevation of an instance at time t (its forcing constituents).
__device__ __forceinline__ double clock_xihat(const InstDesc &I, double t)
{
    double x = 0.0;
    for (int c = 0; c < I.ncon; ++c) x += I.amp[c] * sin(I.omega[c] * t + I.phase[c]);
    return x;
}

// The device clock of an instance for the step about to run: a failed
// instance (non-positive depth or a non-finite value) or one whose step
// budget is spent stops; otherwise the open-sea elevation at the step's two
// stage times is set and the time advanced.
__device__ __forceinline__ void clock_advance(InstDesc &I, int flag)
{
    const int run = I.active && I.steps_left > 0 && flag == 0;
    I.run = run;
    if (!run) return;
    I.xh[0] = clock_xihat(I, I.t);
    I.xh[1] = clock_xihat(I, I.t + I.dt);
    I.t = I.t0 + (double)(I.steps_done + 1) * I.dt;
    I.steps_done += 1;
    I.steps_left -= 1;
}

__global__ void __launch_bounds__(BLOCK) k_batch_clock(InstDesc *inst, const int *flags, int n)
{
    const int i = blockIdx.x * BLOCK + threadIdx.x;
    if (i >= n) return;
    clock_advance(inst[i], flags[i]);
}

// ------------------------------------------------------------ listed elements, every order in one launch
// The kernels of the listed elements take every order in one launch (each
// block runs one order's code; order p's list at a.list + p * lcap, its
// length a.count[p]).  A step graph dispatches its nodes one after another,
// microseconds apart, so one node per stage for all orders ends the stage
// sooner than one node per order.  Block b over the orders lo..PN takes
// order lo + b % (PN - lo + 1) and the (b / (PN - lo + 1))-th run of BLOCK
// list entries (of TEAM entries where a team takes them): the orders are
// interleaved, so the blocks dispatched first hold the heads of every
// order's list.  Lists re-chosen on the device are sized
// for every element and are mostly empty; a block past its list's end leaves
// before it loads anything else (the test is uniform over the block).
template <int PN>
__device__ __forceinline__ int list_order(int lo) { return lo + (int)blockIdx.x % (PN - lo + 1); }
template <int PN>
__device__ __forceinline__ int list_block(int lo) { return (int)blockIdx.x / (PN - lo + 1); }
__device__ __forceinline__ int list_len(const int *count, int p, int lcap)
{
    const int n = count[p];
    return n < lcap ? n : lcap;
}

// Element of entry i of order p's list, or -1 past the list's end.  The
// count is capped at the list's capacity and an entry outside the mesh is
// skipped, so a list is only ever read within its allocation and an entry is
// only ever followed into the element arrays.
template <typename Real>
__device__ __forceinline__ int list_element(const StageArgs<Real> &a, int p, int i, int lcap)
{
    const int n = a.count[p];
    if (i >= (n < lcap ? n : lcap)) return -1;
    const int e = a.list[(size_t)p * (size_t)lcap + (size_t)i];
    return (e >= 0 && e < a.m.ne) ? e : -1;
}

// ---- teams: the listed elements' work shared by the waves of a block
// One thread's evaluation of an order-3 element is thousands of dependent
// instructions, and the few such elements end the stage.  A team block takes
// TEAM list entries, one per lane, and each of its four waves does one part
// of every entry's right-hand side: wave 0 the volume and source terms, wave
// 1 + k the term of local edge k.  Waves 1..3 leave their partial sums in
// LDS; wave 0 adds them in edge order and finishes the element.
// Teams take the short lists (at most TEAM_MAX entries), where the stage
// waits on each element's latency, and every list of a kernel that reaches
// order 3; a long list of a kernel up to order 2 keeps one element per
// thread, which does less work in all.  (One thread per order-3 element needs
// more registers than a lane has, and the one-thread code of the lower orders
// beside the order-3 teams would cost those teams registers.)
constexpr int TEAM = 64;
constexpr int TEAM_ROLES = 4;
constexpr int TEAM_MAX = 16384;

template <int PN>
__device__ __forceinline__ bool list_by_teams(int len) { return PN >= 3 || len <= TEAM_MAX; }

template <int PN, typename Real>
struct TeamLds {
    static constexpr int K = Ord<PN>::K;
    static constexpr bool SPLIT = !std::is_same<Real, double>::value;
    Real L[TEAM_ROLES - 1][3][K][TEAM];
    double W[TEAM_ROLES - 1][SPLIT ? 2 : 1][SPLIT ? K : 1][TEAM];
};

template <int P, int PN, typename Real>
__device__ __forceinline__ void team_put(TeamLds<PN, Real> &X, int role, int lane, const Acc<P, Real> &A)
{
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < Ord<P>::K; ++q) X.L[role - 1][j][q][lane] = A.L[j][q];
    if constexpr (Acc<P, Real>::SPLIT) {
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int q = 0; q < Ord<P>::K; ++q) X.W[role - 1][j][q][lane] = A.W[j][q];
    }
}

// wave 0's sums plus the edge waves' partial sums, in edge order; the FP64
// bathymetry sums of the FP32 path are added to the momentum rows last
template <int P, int PN, typename Real>
__device__ __forceinline__ void team_sum(const TeamLds<PN, Real> &X, int lane, Acc<P, Real> &A)
{
#pragma unroll
    for (int r = 0; r < TEAM_ROLES - 1; ++r) {
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int q = 0; q < Ord<P>::K; ++q) A.L[j][q] += X.L[r][j][q][lane];
        if constexpr (Acc<P, Real>::SPLIT) {
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int q = 0; q < Ord<P>::K; ++q) A.W[j][q] += X.W[r][j][q][lane];
        }
    }
    if constexpr (Acc<P, Real>::SPLIT) {
#pragma unroll
        for (int q = 0; q < Ord<P>::K; ++q) {
            A.L[1][q] += Real(A.W[0][q]);
            A.L[2][q] += Real(A.W[1][q]);
        }
    }
}

// acc += dt * (extra right-hand side) (wave 0's part)
template <int P, typename Real>
__device__ __forceinline__ void team_src(const StageArgs<Real> &a, unsigned e, double dt, Acc<P, Real> &A)
{
    if (!a.src) return;
    const Buf<Real> bS(a.src, 3 * a.m.KS, a.m.stride);
    const Real rdt = Real(dt);
    const unsigned off = e * (unsigned)sizeof(Real);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < Ord<P>::K; ++q) A.L[j][q] = fma(rdt, bS.ld(j * a.m.KS + q, off), A.L[j][q]);
}

// one wave's part (role) of element e's right-hand side, added to A
template <int P, int PN, typename Real>
__device__ __forceinline__ void team_part(int role, const StageArgs<Real> &a, unsigned e, const Buf<Real> &bC,
                                          const Buf<Real> &bU, const Buf<int> &bNb, const Fields<P, Real> &s,
                                          const Geo &G, const double (&hbh)[3], double dt,
                                          const Real (*sR)[Ord<PN>::K][(P > PN ? P : PN) + 1], double xihat,
                                          Acc<P, Real> &A)
{
    switch (role) {
    case 0:
        volume_term<P, Real>(s, hbh, G, a.ph.g, dt, A);
        source_term<P, Real>(s, G, a.ph, dt, A);
        team_src<P, Real>(a, e, dt, A);
        break;
    case 1: edge_one<P, PN, Real, 0>(a.m, e, bC, bU, bNb, s, G, a.ph.g, xihat, dt, sR, A); break;
    case 2: edge_one<P, PN, Real, 1>(a.m, e, bC, bU, bNb, s, G, a.ph.g, xihat, dt, sR, A); break;
    default: edge_one<P, PN, Real, 2>(a.m, e, bC, bU, bNb, s, G, a.ph.g, xihat, dt, sR, A); break;
    }
}

// full stage of listed element e of order P (order-partitioned scheme), one thread
template <int P, int PN, typename Real, int MODE>
__device__ __forceinline__ void full_element(const StageArgs<Real> &a, unsigned e,
                                             const Real (*sR)[Ord<PN>::K][PN + 1], double xihat, double dt)
{
    const MeshView &m = a.m;
    const int KS = m.KS, stride = m.stride;
    const Buf<Real> bC(a.Cin, 3 * KS, stride), bU(a.Uin, 2 * KS, stride);
    const Buf<int> bEv(m.ev, 3, stride), bNb(m.enb, 3, stride);
    const unsigned off = e * (unsigned)sizeof(Real);
    Geo G;
    load_geo(m.vtx, bEv, e * 4u, G);
    double hbh[3];
    hb_modes(G, hbh);
    Fields<P, Real> s;
    load_state<P, Real>(bC, bU, KS, off, s);
    Acc<P, Real> A;
    acc_init<P, Real>(A, s, true);
    element_rhs<P, PN, Real>(a, e, bC, bU, bNb, s, G, hbh, dt, sR, A, xihat);
    finish_stage<P, Real, MODE>(a, e, G, hbh, Ord<P>::K, A.L, a.flag);
}

// the same by a team; live is false on lanes past the list's end, which only
// meet the barrier
template <int P, int PN, typename Real, int MODE>
__device__ __forceinline__ void full_team(const StageArgs<Real> &a, int le, int role,
                                          const Real (*sR)[Ord<PN>::K][PN + 1], TeamLds<PN, Real> &X,
                                          double xihat, double dt)
{
    const MeshView &m = a.m;
    const int KS = m.KS, stride = m.stride, lane = (int)threadIdx.x % TEAM;
    const bool live = le >= 0;
    const unsigned e = live ? (unsigned)le : 0u;
    const Buf<Real> bC(a.Cin, 3 * KS, stride), bU(a.Uin, 2 * KS, stride);
    const Buf<int> bEv(m.ev, 3, stride), bNb(m.enb, 3, stride);
    Geo G;
    double hbh[3];
    Acc<P, Real> A;
    if (live) {
        load_geo(m.vtx, bEv, e * 4u, G);
        hb_modes(G, hbh);
        Fields<P, Real> s;
        load_state<P, Real>(bC, bU, KS, e * (unsigned)sizeof(Real), s);
        acc_init<P, Real>(A, s, role == 0);
        team_part<P, PN, Real>(role, a, e, bC, bU, bNb, s, G, hbh, dt, sR, xihat, A);
        if (role > 0) team_put<P, PN, Real>(X, role, lane, A);
    }
    __syncthreads();
    if (role == 0 && live) {
        team_sum<P, PN, Real>(X, lane, A);
        finish_stage<P, Real, MODE>(a, e, G, hbh, Ord<P>::K, A.L, a.flag);
    }
}

template <int PN, typename Real, int MODE>
__global__ void __launch_bounds__(TEAM * TEAM_ROLES) __attribute__((amdgpu_waves_per_eu(1, 8)))
k_full_all(StageArgs<Real> a, int lo, int lcap)
{
    // beside the base kernel over all elements, these end the stage: their
    // waves issue first on a shared SIMD
    __builtin_amdgcn_s_setprio(2);
    constexpr int NX = PN + 1, KN = Ord<PN>::K;
    __shared__ Real sR[3][KN][NX];
    __shared__ TeamLds<PN, Real> X;
    const int p = list_order<PN>(lo), len = list_len(a.count, p, lcap);
    const bool team = list_by_teams<PN>(len);
    int c = list_block<PN>(lo);
    if (c * (team ? TEAM : BLOCK) >= len) return;
    double xihat = a.xihat, dt = a.dt;
    if (a.inst) {
        if (!a.inst->run) return;   // the step's clock stopped (failure); uniform over the block
        xihat = MODE == MODE_STAGE2 ? a.inst->xh[1] : a.inst->xh[0];
        dt = a.inst->dt;
    }
    load_trace_table<KN, NX, Real>(sR);
    __syncthreads();
    if (team) {
        // one run per block (the grid covers every run, see list_grid)
        const int role = __builtin_amdgcn_readfirstlane((int)threadIdx.x / TEAM);
        const int le = list_element(a, p, c * TEAM + (int)threadIdx.x % TEAM, lcap);
        switch (p) {
        case 0: full_team<0, PN, Real, MODE>(a, le, role, sR, X, xihat, dt); break;
        case 1: if constexpr (PN >= 1) full_team<1, PN, Real, MODE>(a, le, role, sR, X, xihat, dt); break;
        case 2: if constexpr (PN >= 2) full_team<2, PN, Real, MODE>(a, le, role, sR, X, xihat, dt); break;
        case 3: if constexpr (PN >= 3) full_team<3, PN, Real, MODE>(a, le, role, sR, X, xihat, dt); break;
        }
        return;
    }
    // one element per thread
    if constexpr (PN < 3) {
        const int le = list_element(a, p, c * BLOCK + (int)threadIdx.x, lcap);
        if (le < 0) return;
        const unsigned e = (unsigned)le;
        switch (p) {
        case 0: full_element<0, PN, Real, MODE>(a, e, sR, xihat, dt); break;
        case 1: if constexpr (PN >= 1) full_element<1, PN, Real, MODE>(a, e, sR, xihat, dt); break;
        case 2: if constexpr (PN >= 2) full_element<2, PN, Real, MODE>(a, e, sR, xihat, dt); break;
        }
    }
}

// correction of listed element e of order P (order-separated scheme): dt
// times the full right-hand side, minus dt times the base part (rows below
// K(B), the element's and its neighbours' first K(B) modes) in the rows below
// K(B); the base part is evaluated first and kept, negated, in registers
// dt times the correction of listed element e of order P: its full
// right-hand side minus its base one (rows below K(B); the base part reads
// the element's and its neighbours' first K(B) modes); G and hbh are loaded
template <int P, int B, int PN, typename Real>
SWE_HD void corr_value(const StageArgs<Real> &a, unsigned e, const Real (*sR)[Ord<PN>::K][PN + 1],
                       const Real (*sRb)[Ord<B>::K][Ord<B>::NT], double xihat, double dt, Geo &G,
                       double (&hbh)[3], Real (&C)[3][Ord<P>::K])
{
    constexpr int K = Ord<P>::K, KB = Ord<B>::K;
    const MeshView &m = a.m;
    const int KS = m.KS, stride = m.stride;
    const Buf<Real> bC(a.Cin, 3 * KS, stride), bU(a.Uin, 2 * KS, stride);
    const Buf<int> bEv(m.ev, 3, stride), bNb(m.enb, 3, stride);
    const unsigned off = e * (unsigned)sizeof(Real);
    load_geo(m.vtx, bEv, e * 4u, G);
    hb_modes(G, hbh);
    Real minus_base[3][KB];
    {
        Fields<B, Real> sb;
        load_state<B, Real>(bC, bU, KS, off, sb);
        Acc<B, Real> Ab;
        acc_init<B, Real>(Ab, sb, false);
        element_rhs<B, B, Real>(a, e, bC, bU, bNb, sb, G, hbh, dt, sRb, Ab, xihat);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int q = 0; q < KB; ++q) minus_base[j][q] = -Ab.L[j][q];
    }
    Fields<P, Real> s;
    load_state<P, Real>(bC, bU, KS, off, s);
    Acc<P, Real> A;
    acc_init<P, Real>(A, s, false);
    element_rhs<P, PN, Real>(a, e, bC, bU, bNb, s, G, hbh, dt, sR, A, xihat);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < K; ++q) {
            Real v = A.L[j][q];
            if (q < KB) v += minus_base[j][q];
            C[j][q] = v;
        }
}

// the correction of listed element e stored in Lc (for the epilogue)
template <int P, int B, int PN, typename Real>
SWE_HD void corr_element(const StageArgs<Real> &a, unsigned e,
                                             const Real (*sR)[Ord<PN>::K][PN + 1],
                                             const Real (*sRb)[Ord<B>::K][Ord<B>::NT], double xihat, double dt)
{
    constexpr int K = Ord<P>::K;
    const int KS = a.m.KS, stride = a.m.stride;
    const Buf<Real> bL(a.Lc, 3 * KS, stride);
    const unsigned off = e * (unsigned)sizeof(Real);
    Geo G;
    double hbh[3];
    Real C[3][K];
    corr_value<P, B, PN, Real>(a, e, sR, sRb, xihat, dt, G, hbh, C);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < K; ++q) bL.st(j * KS + q, off, C[j][q]);
}

// The epilogue joined into the correction kernel (a.finish set: the base
// pass has run before it, not beside it): stage value = (the base partial
// value in Lb, or c for modes >= K(B)) + the correction C, the same sum the
// epilogue forms, then the listed element's stage finished
template <int P, int B, typename Real>
__device__ __forceinline__ void join_finish(const StageArgs<Real> &a, unsigned e, const Geo &G,
                                            const double (&hbh)[3], Real (&C)[3][Ord<P>::K])
{
    constexpr int K = Ord<P>::K, KB = Ord<B>::K;
    const int KS = a.m.KS, stride = a.m.stride;
    const Buf<Real> bC(a.Cin, 3 * KS, stride), bB(a.Lb, 3 * KB, stride);
    const unsigned off = e * (unsigned)sizeof(Real);
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < K; ++q) C[j][q] = (q < KB ? bB.ld(j * KB + q, off) : bC.ld(j * KS + q, off)) + C[j][q];
    if (a.finish == MODE_STAGE2)
        finish_stage<P, Real, MODE_STAGE2>(a, e, G, hbh, K, C, a.flag);
    else
        finish_stage<P, Real, MODE_STAGE1>(a, e, G, hbh, K, C, a.flag);
}

// correction of listed element e of order P by a team: each wave's part of
// the full right-hand side minus its part of the base one (rows below K(B);
// the base part reads the element's and its neighbours' first K(B) modes),
// summed by wave 0, which stores dt times the correction
template <int P, int B, int PN, typename Real>
__device__ __forceinline__ void corr_team(const StageArgs<Real> &a, int le, int role,
                                          const Real (*sR)[Ord<PN>::K][PN + 1],
                                          const Real (*sRb)[Ord<B>::K][Ord<B>::NT], TeamLds<PN, Real> &X,
                                          double xihat, double dt)
{
    constexpr int K = Ord<P>::K, KB = Ord<B>::K;
    const MeshView &m = a.m;
    const int KS = m.KS, stride = m.stride, lane = (int)threadIdx.x % TEAM;
    const bool live = le >= 0;
    const unsigned e = live ? (unsigned)le : 0u;
    const unsigned off = e * (unsigned)sizeof(Real);
    const Buf<Real> bC(a.Cin, 3 * KS, stride), bU(a.Uin, 2 * KS, stride);
    const Buf<int> bEv(m.ev, 3, stride), bNb(m.enb, 3, stride);
    Acc<P, Real> A;
    Geo G;
    double hbh[3];
    // wave 0 of a kernel that finishes the stage (a.finish) fetches what the
    // join needs before its volume work, so the loads overlap it: the base
    // part (c itself above K(B)) and, in the second stage, c^n
    const bool join = role == 0 && a.finish;
    Real Jb[3][K], Jn[3][K];
    if (live) {
        load_geo(m.vtx, bEv, e * 4u, G);
        hb_modes(G, hbh);
        Fields<P, Real> s;
        load_state<P, Real>(bC, bU, KS, off, s);
        if (join) {
            const Buf<Real> bB(a.Lb, 3 * KB, stride), bN(a.Cn, 3 * KS, stride);
#pragma unroll
            for (int q = 0; q < K; ++q) {
                Jb[0][q] = q < KB ? bB.ld(0 * KB + q, off) : s.xi[q];
                Jb[1][q] = q < KB ? bB.ld(1 * KB + q, off) : s.U[q];
                Jb[2][q] = q < KB ? bB.ld(2 * KB + q, off) : s.V[q];
            }
            if (a.finish == MODE_STAGE2) {
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int q = 0; q < K; ++q) Jn[j][q] = bN.ld(j * KS + q, off);
            }
        }
        {
            Fields<B, Real> sb;
#pragma unroll
            for (int q = 0; q < KB; ++q) {
                sb.xi[q] = s.xi[q]; sb.U[q] = s.U[q]; sb.V[q] = s.V[q]; sb.u[q] = s.u[q]; sb.v[q] = s.v[q];
            }
            Acc<B, Real> Ab;
            acc_init<B, Real>(Ab, sb, false);
            team_part<B, B, Real>(role, a, e, bC, bU, bNb, sb, G, hbh, dt, sRb, xihat, Ab);
            acc_init<P, Real>(A, s, false);
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int q = 0; q < KB; ++q) A.L[j][q] = -Ab.L[j][q];
            if constexpr (Acc<P, Real>::SPLIT) {
#pragma unroll
                for (int j = 0; j < 2; ++j)
#pragma unroll
                    for (int q = 0; q < KB; ++q) A.W[j][q] = -Ab.W[j][q];
            }
        }
        team_part<P, PN, Real>(role, a, e, bC, bU, bNb, s, G, hbh, dt, sR, xihat, A);
        if (role > 0) team_put<P, PN, Real>(X, role, lane, A);
    }
    __syncthreads();
    if (role == 0 && live) {
        team_sum<P, PN, Real>(X, lane, A);
        if (join) {
            // the epilogue's sum and, in the second stage, the RK combine, in
            // the expressions of join_finish and finish_stage (bit for bit)
#pragma unroll
            for (int j = 0; j < 3; ++j)
#pragma unroll
                for (int q = 0; q < K; ++q) A.L[j][q] = Jb[j][q] + A.L[j][q];
            if (a.finish == MODE_STAGE2) {
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int q = 0; q < K; ++q) A.L[j][q] = Real(0.5) * Jn[j][q] + Real(0.5) * A.L[j][q];
            }
            finish_stage<P, Real, MODE_STAGE1>(a, e, G, hbh, K, A.L, a.flag);
            return;
        }
        const Buf<Real> bL(a.Lc, 3 * KS, stride);
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int q = 0; q < K; ++q) bL.st(j * KS + q, off, A.L[j][q]);
    }
}

// correction of listed element e by one thread: stored for the epilogue, or
// joined with the base part and the stage finished (a.finish)
template <int P, int B, int PN, typename Real>
__device__ __forceinline__ void corr_thread(const StageArgs<Real> &a, unsigned e,
                                            const Real (*sR)[Ord<PN>::K][PN + 1],
                                            const Real (*sRb)[Ord<B>::K][Ord<B>::NT], double xihat, double dt)
{
    if (!a.finish) {
        corr_element<P, B, PN, Real>(a, e, sR, sRb, xihat, dt);
        return;
    }
    Geo G;
    double hbh[3];
    Real C[3][Ord<P>::K];
    corr_value<P, B, PN, Real>(a, e, sR, sRb, xihat, dt, G, hbh, C);
    join_finish<P, B, Real>(a, e, G, hbh, C);
}

template <int B, int PN, typename Real>
__global__ void __launch_bounds__(TEAM * TEAM_ROLES) __attribute__((amdgpu_waves_per_eu(1, 8)))
k_corr_all(StageArgs<Real> a, double dt, int lcap)
{
    __builtin_amdgcn_s_setprio(2);   // as in k_full_all
    constexpr int KB = Ord<B>::K, NTB = Ord<B>::NT;
    constexpr int KN = Ord<PN>::K, NX = PN + 1;
    __shared__ Real sR[3][KN][NX];
    __shared__ Real sRb[3][KB][NTB];
    __shared__ TeamLds<PN, Real> X;
    const int p = list_order<PN>(B), len = list_len(a.count, p, lcap);
    const bool team = list_by_teams<PN>(len);
    int c = list_block<PN>(B);
    if (c * (team ? TEAM : BLOCK) >= len) return;
    double xihat = a.xihat;
    if (a.inst) {
        // the clock of a replayed step lives on the device
        if (!a.inst->run) return;   // the step's clock stopped (failure); uniform over the block
        xihat = a.inst->xh[a.stage];
        dt = a.inst->dt;
    }
    load_trace_table<KN, NX, Real>(sR);
    load_trace_table<KB, NTB, Real>(sRb);
    __syncthreads();
    if (team) {   // as in k_full_all
        const int role = __builtin_amdgcn_readfirstlane((int)threadIdx.x / TEAM);
        const int le = list_element(a, p, c * TEAM + (int)threadIdx.x % TEAM, lcap);
        switch (p) {
        case 0: if constexpr (B <= 0) corr_team<0, B, PN, Real>(a, le, role, sR, sRb, X, xihat, dt); break;
        case 1: if constexpr (B <= 1 && PN >= 1) corr_team<1, B, PN, Real>(a, le, role, sR, sRb, X, xihat, dt); break;
        case 2: if constexpr (B <= 2 && PN >= 2) corr_team<2, B, PN, Real>(a, le, role, sR, sRb, X, xihat, dt); break;
        case 3: if constexpr (B <= 3 && PN >= 3) corr_team<3, B, PN, Real>(a, le, role, sR, sRb, X, xihat, dt); break;
        }
        return;
    }
    if constexpr (PN < 3) {
        const int le = list_element(a, p, c * BLOCK + (int)threadIdx.x, lcap);
        if (le < 0) return;
        const unsigned e = (unsigned)le;
        switch (p) {
        case 0: if constexpr (B <= 0) corr_thread<0, B, PN, Real>(a, e, sR, sRb, xihat, dt); break;
        case 1: if constexpr (B <= 1 && PN >= 1) corr_thread<1, B, PN, Real>(a, e, sR, sRb, xihat, dt); break;
        case 2: if constexpr (B <= 2 && PN >= 2) corr_thread<2, B, PN, Real>(a, e, sR, sRb, xihat, dt); break;
        }
    }
}

// The same correction on the host (the heterogeneous stage): the listed
// elements [e0, e1) of every order, split over nthreads CPU threads; the
// arguments point at host copies of the mesh and of the stage's input state,
// and the correction goes to a host copy of Lc.
template <int B, int PN, typename Real>
void host_corr_t(const StageArgs<Real> &a, double dt, const signed char *order, int e0, int e1, int nthreads)
{
    constexpr int KN = Ord<PN>::K, NX = PN + 1, KB = Ord<B>::K, NTB = Ord<B>::NT;
    Real sR[3][KN][NX], sRb[3][KB][NTB];
    for (int k = 0; k < 3; ++k) {
        for (int n = 0; n < KN; ++n)
            for (int c = 0; c < NX; ++c) sR[k][n][c] = Real(TR[k][n][c]);
        for (int n = 0; n < KB; ++n)
            for (int c = 0; c < NTB; ++c) sRb[k][n][c] = Real(TR[k][n][c]);
    }
    auto work = [&](int lo, int hi) {
        for (int e = lo; e < hi; ++e) {
            const unsigned ue = (unsigned)e;
            switch (order[e]) {
            case 0: if constexpr (B <= 0) corr_element<0, B, PN, Real>(a, ue, sR, sRb, a.xihat, dt); break;
            case 1: if constexpr (B <= 1 && PN >= 1) corr_element<1, B, PN, Real>(a, ue, sR, sRb, a.xihat, dt); break;
            case 2: if constexpr (B <= 2 && PN >= 2) corr_element<2, B, PN, Real>(a, ue, sR, sRb, a.xihat, dt); break;
            case 3: if constexpr (B <= 3 && PN >= 3) corr_element<3, B, PN, Real>(a, ue, sR, sRb, a.xihat, dt); break;
            }
        }
    };
    const int n = e1 - e0;
    if (n <= 0) return;
    const int nt = std::max(1, std::min(nthreads, (n + 63) / 64));
    std::vector<std::thread> pool;
    for (int t = 1; t < nt; ++t)
        pool.emplace_back(work, e0 + (int)((int64_t)n * t / nt), e0 + (int)((int64_t)n * (t + 1) / nt));
    work(e0, e0 + (int)((int64_t)n / nt));
    for (auto &th : pool) th.join();
}

// epilogue of listed element e of order P (order-separated scheme): stage
// value = (base partial value, or c for modes >= K(B)) + correction
template <int P, typename Real, int MODE>
__device__ __forceinline__ void epi_element(const StageArgs<Real> &a, unsigned e, int KB)
{
    constexpr int K = Ord<P>::K;
    const MeshView &m = a.m;
    const int KS = m.KS, stride = m.stride;
    const Buf<Real> bC(a.Cin, 3 * KS, stride), bL(a.Lc, 3 * KS, stride), bB(a.Lb, 3 * KB, stride);
    const Buf<int> bEv(m.ev, 3, stride);
    const unsigned off = e * (unsigned)sizeof(Real);
    Geo G;
#pragma unroll
    for (int v = 0; v < 3; ++v) G.h[v] = m.vtx[(unsigned)bEv.ld(v, e * 4u)].z;
    double hbh[3];
    hb_modes(G, hbh);
    Real L[3][K];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int q = 0; q < K; ++q)
            L[j][q] = (q < KB ? bB.ld(j * KB + q, off) : bC.ld(j * KS + q, off)) + bL.ld(j * KS + q, off);
    finish_stage<P, Real, MODE>(a, e, G, hbh, K, L, a.flag);
}

template <int PN, typename Real, int MODE>
__global__ void __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(1, 8)))
k_epi_all(StageArgs<Real> a, int KB, int lo, int lcap)
{
    const int p = list_order<PN>(lo), first = list_block<PN>(lo) * BLOCK;
    if (first >= list_len(a.count, p, lcap)) return;
    const int le = list_element(a, p, first + (int)threadIdx.x, lcap);
    if (le < 0) return;
    const unsigned e = (unsigned)le;
    if (a.inst && !a.inst->run) return;   // the step's clock stopped (failure)
    switch (p) {
    case 0: epi_element<0, Real, MODE>(a, e, KB); break;
    case 1: if constexpr (PN >= 1) epi_element<1, Real, MODE>(a, e, KB); break;
    case 2: if constexpr (PN >= 2) epi_element<2, Real, MODE>(a, e, KB); break;
    case 3: if constexpr (PN >= 3) epi_element<3, Real, MODE>(a, e, KB); break;
    }
}

// ------------------------------------------------------------ p-adaptivity
// Indicator (stand-in for the paper's JRL indicator, which its text only
// cites): the largest jump of the P1 part of xi at the edge midpoints; land
// edges contribute 0, open edges compare with xi_hat(t).  New order: p_hi if
// I >= tau, one less for each further factor 10 below tau, never below p_lo.
template <typename Real>
__device__ __forceinline__ void indicator_element(const MeshView &m, const Buf<Real> &bC, unsigned e, double xihat,
                                                  double tau, int p_lo, int p_hi, double *I_out, signed char *p_new)
{
    const Buf<int> bNb(m.enb, 3, m.stride);
    const unsigned off = e * (unsigned)sizeof(Real);
    const double x0 = bC.ld(0, off), x1 = bC.ld(1, off), x2 = bC.ld(2, off);
    const unsigned nbk_all = m.enbk[e];
    double I = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double own = TPMID[k][0] * x0 + TPMID[k][1] * x1 + TPMID[k][2] * x2;
        const int nb = bNb.ld(k, e * 4u);
        double other = own;
        if (nb >= 0) {
            const int kk = (nbk_all >> (2 * k)) & 3;
            const unsigned on = (unsigned)nb * (unsigned)sizeof(Real);
            const double y0 = bC.ld(0, on), y1 = bC.ld(1, on), y2 = bC.ld(2, on);
            other = TPMID[kk][0] * y0 + TPMID[kk][1] * y1 + TPMID[kk][2] * y2;
        } else if (nb == NB_OPEN) {
            other = xihat;
        }
        const double j = fabs(own - other);
        I = j > I ? j : I;
    }
    if (I_out) I_out[e] = I;
    if (p_new) {
        int pn = p_lo;
        double thr = tau;
        for (int pp = p_hi; pp > p_lo; --pp) {
            if (I >= thr) { pn = pp; break; }
            thr *= 0.1;
        }
        p_new[e] = (signed char)pn;
    }
}

template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_indicator(StageArgs<Real> a, double tau, int p_lo, int p_hi,
                                                     double *I_out, signed char *p_new)
{
    const MeshView &m = a.m;
    if (a.cntw && blockIdx.x == 0 && threadIdx.x < 4) a.cntw[threadIdx.x] = 0;   // list counts of the next pass
    const unsigned e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= (unsigned)m.ne) return;
    const Buf<Real> bC(a.Cin, 3 * m.KS, m.stride);
    // in a step graph the clock advances in the order update after this
    // kernel, so the step's start time is still the clock's time
    indicator_element<Real>(m, bC, e, a.inst ? clock_xihat(*a.inst, a.inst->t) : a.xihat, tau, p_lo, p_hi, I_out,
                            p_new);
}

// Apply the new order of element e: drop modes above K(p_new) from every state
// buffer and re-solve u if the order changed; whether the element is listed
// (its order or a neighbour's above p_base) goes to *listed.
template <int PM, typename Real>
__device__ __forceinline__ int apply_element(const StageArgs<Real> &a, unsigned e, const signed char *p_new,
                                             signed char *p_cur, int p_base, bool *listed)
{
    constexpr int K = Ord<PM>::K;
    const MeshView &m = a.m;
    const int KS = m.KS, stride = m.stride;
    const unsigned off = e * (unsigned)sizeof(Real);
    const int pn = p_new[e];
    const int po = p_cur[e];
    const Buf<int> bNb(m.enb, 3, stride);
    bool l = pn > p_base;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int nb = bNb.ld(k, e * 4u);
        if (nb >= 0 && p_new[nb] > p_base) l = true;
    }
    *listed = l;
    if (pn != po) {
        const int Kn = KOFP[pn];
        Buf<Real> b0(a.Cout, 3 * KS, stride), b1(a.Calt, 3 * KS, stride);
        Buf<Real> u1(a.Ualt, 2 * KS, stride);
        Real xi[K], U[K], V[K];
#pragma unroll
        for (int q = 0; q < K; ++q) {
            const bool keep = q < Kn;
            xi[q] = keep ? b0.ld(0 * KS + q, off) : Real(0);
            U[q] = keep ? b0.ld(1 * KS + q, off) : Real(0);
            V[q] = keep ? b0.ld(2 * KS + q, off) : Real(0);
            if (!keep) {
#pragma unroll
                for (int j = 0; j < 3; ++j) { b0.st(j * KS + q, off, Real(0)); b1.st(j * KS + q, off, Real(0)); }
                u1.st(0 * KS + q, off, Real(0));
                u1.st(1 * KS + q, off, Real(0));
            }
        }
        Geo G;
#pragma unroll
        for (int v = 0; v < 3; ++v) G.h[v] = m.vtx[(unsigned)Buf<int>(m.ev, 3, stride).ld(v, e * 4u)].z;
        double hbh[3];
        hb_modes(G, hbh);
        Real u[K], v[K];
        solve_u<PM, Real>(xi, U, V, hbh, Kn, u, v);
        Buf<Real> bu(a.Uout, 2 * KS, stride);
#pragma unroll
        for (int q = 0; q < K; ++q) {
            bu.st(0 * KS + q, off, u[q]);
            bu.st(1 * KS + q, off, v[q]);
        }
        p_cur[e] = (signed char)pn;
    }
    return pn;
}

// Apply the new orders of a context's elements, flag elements that need a
// correction and append them to the list of their order (one atomic per
// wave and order).
template <int PM, typename Real>
__global__ void __launch_bounds__(BLOCK) k_apply_order(StageArgs<Real> a, const signed char *p_new,
                                                       signed char *p_cur, int p_base, int lcap, InstDesc *clock,
                                                       const int *flag)
{
    const unsigned e = blockIdx.x * BLOCK + threadIdx.x;
    // a step graph's clock (no other thread of this kernel reads the instance)
    if (clock && e == 0) clock_advance(*clock, flag[0]);
    const bool live = e < (unsigned)a.m.ne;
    int pn = 0;
    bool listed = false;
    if (live) {
        pn = apply_element<PM, Real>(a, e, p_new, p_cur, p_base, &listed);
        a.inlist[e] = listed ? 1 : 0;
    }
    // wave-aggregated append to the list of order pn
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int p = 0; p < 4; ++p) {
        const bool mine = live && listed && pn == p;
        const unsigned long long mask = __ballot(mine);
        if (mask == 0ull) continue;
        const int leader = __ffsll((long long)mask) - 1;
        int base = 0;
        if (lane == leader) base = atomicAdd(&a.cntw[p], __popcll(mask));
        base = __shfl(base, leader);
        if (mine) {
            // base + rank < lcap: each element is appended at most once per update
            const int rank = __popcll(mask & ((1ull << lane) - 1ull));
            if (base + rank < lcap) a.listw[(size_t)p * (size_t)lcap + (size_t)(base + rank)] = (int)e;
        }
    }
}

// The order update of the indicator-driven members of a batch, over 256-element
// tiles of their pool (every such member runs the fused scheme: its elements'
// own orders mask the stage, no lists).  Tile lists and instance scalars as
// for the batch stage kernels; instances whose clock stopped are skipped.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_batch_indicator(BatchArgs b)
{
    const int nt = b.natiles[0];
    const int x = (int)(blockIdx.x & 7u), i = (int)(blockIdx.x >> 3);
    const int lo = (int)(((long long)nt * x) >> 3), hi = (int)(((long long)nt * (x + 1)) >> 3);
    const int t = lo + i;
    if (t >= hi) return;
    const int2 tile = b.atiles[t];
    const InstDesc &I = b.inst[tile.x];
    if (!I.run) return;
    const unsigned e = (unsigned)tile.y + threadIdx.x;
    if (e >= (unsigned)(I.first + I.ne)) return;
    MeshView m{};
    m.stride = b.pool.cap;
    m.KS = (I.order + 1) * (I.order + 2) / 2;
    m.vtx = b.vtx;
    m.ev = b.pool.ev;
    m.enb = b.pool.nb;
    m.enbk = b.pool.nbk;
    const Buf<Real> bC(static_cast<const Real *>(b.pool.C0), 3 * m.KS, m.stride);
    indicator_element<Real>(m, bC, e, I.xh[0], I.tau, I.p_lo, I.order, nullptr, b.pool.pnew);
}

template <int PM, typename Real>
__global__ void __launch_bounds__(BLOCK) k_batch_apply(BatchArgs b)
{
    const int nt = b.natiles[0];
    const int x = (int)(blockIdx.x & 7u), i = (int)(blockIdx.x >> 3);
    const int lo = (int)(((long long)nt * x) >> 3), hi = (int)(((long long)nt * (x + 1)) >> 3);
    const int t = lo + i;
    if (t >= hi) return;
    const int2 tile = b.atiles[t];
    const InstDesc &I = b.inst[tile.x];
    if (!I.run) return;
    const unsigned e = (unsigned)tile.y + threadIdx.x;
    if (e >= (unsigned)(I.first + I.ne)) return;
    StageArgs<Real> a{};   // no lists: the fused scheme masks by the elements' own orders
    a.m.stride = b.pool.cap;
    a.m.KS = Ord<PM>::K;
    a.m.vtx = b.vtx;
    a.m.ev = b.pool.ev;
    a.m.enb = b.pool.nb;
    a.m.enbk = b.pool.nbk;
    a.Cout = static_cast<Real *>(b.pool.C0);
    a.Calt = static_cast<Real *>(b.pool.C1);
    a.Uout = static_cast<Real *>(b.pool.U0);
    a.Ualt = static_cast<Real *>(b.pool.U1);
    bool listed = false;
    (void)apply_element<PM, Real>(a, e, b.pool.pnew, b.pool.ep, I.p_lo, &listed);
}

// ------------------------------------------------------------ minimum depth control
// After a stage (the paper's minimum depth control, a kernel of its code that
// it does not define; this is the reading): an element whose total depth
// H = xi + h_b is below h_min at one of its vertices or edge midpoints has the
// deviation of H from its element mean scaled by
//   theta = (mean H - h_min) / (mean H - min H)   (0 when mean H <= h_min),
// keeping the mean (the mass), and the momentum's deviation from its mean is
// scaled by the same theta.  h_b is fixed, so xi takes the scaled deviation
// of H minus that of h_b (its modes 1 and 2).  The element's velocity is then
// solved again.  Order-0 elements have no mode to scale.
template <int PM, typename Real>
__global__ void __launch_bounds__(BLOCK) k_depth_limit(StageArgs<Real> a, double h_min)
{
    constexpr int K = Ord<PM>::K;
    const MeshView &m = a.m;
    const unsigned e = blockIdx.x * BLOCK + threadIdx.x;
    if (e >= (unsigned)m.ne) return;
    if (a.inst && !a.inst->run) return;   // the step's clock stopped (failure)
    const int p = m.ep ? (int)m.ep[e] : PM;
    if (p < 1) return;
    const int Ke = KOFP[p];
    const int KS = m.KS, stride = m.stride;
    const unsigned off = e * (unsigned)sizeof(Real);
    const Buf<Real> bC(a.Cout, 3 * KS, stride);
    Geo G;
#pragma unroll
    for (int v = 0; v < 3; ++v) G.h[v] = m.vtx[(unsigned)Buf<int>(m.ev, 3, stride).ld(v, e * 4u)].z;
    Real xi[K];
#pragma unroll
    for (int q = 0; q < K; ++q) xi[q] = q < Ke ? bC.ld(q, off) : Real(0);
    const double hbm = (G.h[0] + G.h[1] + G.h[2]) * (1.0 / 3.0);
    const double Hm = SQRT2 * double(xi[0]) + hbm;
    // check points: vertex j < 3, the midpoint of edge j - 3 (it joins
    // vertices j - 2 and j - 1, modulo 3) for j >= 3
    double Hlow = HUGE_VAL;
#pragma unroll
    for (int j = 0; j < 6; ++j) {
        double x = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) x = fma(TCHK[j][q], double(xi[q]), x);
        const double hb = j < 3 ? G.h[j] : 0.5 * (G.h[(j - 2) % 3] + G.h[(j - 1) % 3]);
        Hlow = fmin(Hlow, x + hb);
    }
    if (!(Hlow < h_min)) return;
    const double theta = Hm > h_min ? (Hm - h_min) / (Hm - Hlow) : 0.0;
    double hbh[3];
    hb_modes(G, hbh);
    const Buf<Real> bU(a.Uout, 2 * KS, stride);
    Real U[K], V[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        U[q] = q < Ke ? bC.ld(KS + q, off) : Real(0);
        V[q] = q < Ke ? bC.ld(2 * KS + q, off) : Real(0);
    }
#pragma unroll
    for (int q = 1; q < K; ++q) {
        if (q >= Ke) continue;
        xi[q] = Real(q < 3 ? theta * double(xi[q]) + (theta - 1.0) * hbh[q] : theta * double(xi[q]));
        U[q] = Real(theta * double(U[q]));
        V[q] = Real(theta * double(V[q]));
        bC.st(q, off, xi[q]);
        bC.st(KS + q, off, U[q]);
        bC.st(2 * KS + q, off, V[q]);
    }
    Real u[K], v[K];
    solve_u<PM, Real>(xi, U, V, hbh, Ke, u, v);
#pragma unroll
    for (int q = 0; q < K; ++q) {
        if (q >= Ke) continue;
        bU.st(q, off, u[q]);
        bU.st(KS + q, off, v[q]);
    }
}

template <int P, typename Real>
__global__ void __launch_bounds__(BLOCK) k_usolve(StageArgs<Real> a)
{
    constexpr int K = Ord<P>::K;
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    const MeshView &m = a.m;
    if (e >= m.ne) return;
    const int KS = m.KS, stride = m.stride;
    Geo G;
#pragma unroll
    for (int v = 0; v < 3; ++v) G.h[v] = m.vtx[m.ev[v * stride + e]].z;
    double hbh[3];
    hb_modes(G, hbh);
    const int Ke = a.mixed ? KOFP[m.ep[e]] : K;
    Real xi[K], U[K], V[K], u[K], v[K];
#pragma unroll
    for (int q = 0; q < K; ++q) {
        xi[q] = a.Cin[(0 * KS + q) * stride + e];
        U[q] = a.Cin[(1 * KS + q) * stride + e];
        V[q] = a.Cin[(2 * KS + q) * stride + e];
    }
    solve_u<P, Real>(xi, U, V, hbh, Ke, u, v);
#pragma unroll
    for (int q = 0; q < K; ++q) {
        a.Uout[(0 * KS + q) * stride + e] = u[q];
        a.Uout[(1 * KS + q) * stride + e] = v[q];
    }
}

// Mass: sum_e int xi = sum_e xi_hat_0 |det B_e| / sqrt(2), fixed-order tree.
template <typename Real>
__global__ void __launch_bounds__(BLOCK) k_mass_partial(MeshView m, const Real *C, double *partial)
{
    __shared__ double red[BLOCK];
    const int e = blockIdx.x * BLOCK + threadIdx.x;
    double v = 0.0;
    if (e < m.ne) {
        Geo G;
        load_geo(m.vtx, Buf<int>(m.ev, 3, m.stride), (unsigned)e * 4u, G);
        v = double(C[e]) * G.det * (1.0 / SQRT2);
    }
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(BLOCK) k_mass_final(const double *partial, int n, double *out)
{
    __shared__ double red[BLOCK];
    double v = 0.0;
    for (int i = threadIdx.x; i < n; i += BLOCK) v += partial[i];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int w = BLOCK / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0];
}

template <int P, typename Real, bool SEP>
hipError_t stage_p(int mode, const void *args, Sink &s)
{
    StageArgs<Real> a = *static_cast<const StageArgs<Real> *>(args);
    if (a.m.ne <= 0) return hipSuccess;
    const int nb = (a.m.ne + BLOCK - 1) / BLOCK;
    const dim3 grid(a.blocks > 0 && a.blocks < nb ? a.blocks : nb), block(BLOCK);
    void *kargs[] = {&a};
    const void *fn = mode == MODE_RHS      ? reinterpret_cast<const void *>(&k_stage<P, Real, MODE_RHS, false>)
                     : mode == MODE_STAGE1 ? reinterpret_cast<const void *>(&k_stage<P, Real, MODE_STAGE1, SEP>)
                                           : reinterpret_cast<const void *>(&k_stage<P, Real, MODE_STAGE2, SEP>);
    return emit(s, fn, grid, block, kargs);
}

template <typename Real>
hipError_t stage_r(int p, int mode, bool sep, const void *args, Sink &s)
{
    if (sep) {
        switch (p) {
        case 0: return stage_p<0, Real, true>(mode, args, s);
        case 1: return stage_p<1, Real, true>(mode, args, s);
        case 2: return stage_p<2, Real, true>(mode, args, s);
        }
        return hipErrorInvalidValue;
    }
    switch (p) {
    case 0: return stage_p<0, Real, false>(mode, args, s);
    case 1: return stage_p<1, Real, false>(mode, args, s);
    case 2: return stage_p<2, Real, false>(mode, args, s);
    case 3: return stage_p<3, Real, false>(mode, args, s);
    }
    return hipErrorInvalidValue;
}

template <int P, typename Real>
hipError_t usolve_p(const void *args, hipStream_t s)
{
    const StageArgs<Real> &a = *static_cast<const StageArgs<Real> *>(args);
    if (a.m.ne <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_usolve<P, Real>), dim3((a.m.ne + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, a);
    return hipGetLastError();
}

template <typename Real>
hipError_t usolve_r(int p, const void *args, hipStream_t s)
{
    switch (p) {
    case 0: return usolve_p<0, Real>(args, s);
    case 1: return usolve_p<1, Real>(args, s);
    case 2: return usolve_p<2, Real>(args, s);
    case 3: return usolve_p<3, Real>(args, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t emit(Sink &k, const void *fn, dim3 grid, dim3 block, void **args)
{
    if (!k.g) return hipLaunchKernel(fn, grid, block, args, 0, k.s);
    hipKernelNodeParams prm{};
    prm.func = const_cast<void *>(fn);
    prm.gridDim = grid;
    prm.blockDim = block;
    prm.sharedMemBytes = 0;
    prm.kernelParams = args;      // copied into the node
    prm.extra = nullptr;
    hipGraphNode_t node = nullptr;
    const hipError_t e = hipGraphAddKernelNode(&node, k.g, k.ndep ? k.dep : nullptr, (size_t)k.ndep, &prm);
    if (e == hipSuccess) {
        k.dep[0] = node;
        k.ndep = 1;
    }
    return e;
}

hipError_t launch_stage(int p, bool fp32, int mode, bool sep, const void *args, Sink &k)
{
    return fp32 ? stage_r<float>(p, mode, sep, args, k) : stage_r<double>(p, mode, sep, args, k);
}

template <int P, typename Real>
hipError_t stage_sh_p(int mode, const void *args, const unsigned *items, const int *item_off, Sink &k)
{
    StageArgs<Real> a = *static_cast<const StageArgs<Real> *>(args);
    if (a.m.ne <= 0) return hipSuccess;
    void *kargs[] = {&a, &items, &item_off};
    const void *fn = mode == MODE_RHS      ? reinterpret_cast<const void *>(&k_stage_sh<P, Real, MODE_RHS>)
                     : mode == MODE_STAGE1 ? reinterpret_cast<const void *>(&k_stage_sh<P, Real, MODE_STAGE1>)
                                           : reinterpret_cast<const void *>(&k_stage_sh<P, Real, MODE_STAGE2>);
    const int nb = (a.m.ne + BLOCK - 1) / BLOCK;
    return emit(k, fn, dim3(a.blocks > 0 && a.blocks < nb ? a.blocks : nb), dim3(BLOCK), kargs);
}

// Order 0 has too little work per edge for the sharing to pay for the LDS
// staging and the barriers.
bool stage_sh_supported(int p, bool fp32)
{
    (void)fp32;
    return p >= 1 && p <= 3;
}

hipError_t launch_stage_sh(int p, bool fp32, int mode, const void *args, const unsigned *items, const int *item_off,
                           Sink &k)
{
    if (fp32) {
        switch (p) {
        case 0: return stage_sh_p<0, float>(mode, args, items, item_off, k);
        case 1: return stage_sh_p<1, float>(mode, args, items, item_off, k);
        case 2: return stage_sh_p<2, float>(mode, args, items, item_off, k);
        case 3: return stage_sh_p<3, float>(mode, args, items, item_off, k);
        }
    } else {
        switch (p) {
        case 0: return stage_sh_p<0, double>(mode, args, items, item_off, k);
        case 1: return stage_sh_p<1, double>(mode, args, items, item_off, k);
        case 2: return stage_sh_p<2, double>(mode, args, items, item_off, k);
        case 3: return stage_sh_p<3, double>(mode, args, items, item_off, k);
        }
    }
    return hipErrorInvalidValue;
}

hipError_t launch_stage(int p, bool fp32, int mode, bool sep, const void *args, hipStream_t s)
{
    Sink k;
    k.s = s;
    return launch_stage(p, fp32, mode, sep, args, k);
}

// Blocks per order of a list kernel whose longest possible list fills nblk
// runs of BLOCK entries: a kernel that reaches order 3 takes every list in
// TEAM-entry runs (4 nblk blocks); below order 3 a block takes a run of BLOCK
// entries (nblk blocks) or, for a list of at most TEAM_MAX entries, a run of
// TEAM entries (at most TEAM_MAX / TEAM blocks).  Lists re-chosen on the
// device are mostly empty, and each block costs a dispatch even when it
// finds nothing to do: no more blocks than these.
int list_grid(int nblk, int pn)
{
    const int runs = nblk * (BLOCK / TEAM);
    if (pn >= 3) return runs;
    const int teams = runs < TEAM_MAX / TEAM ? runs : TEAM_MAX / TEAM;
    return nblk > teams ? nblk : teams;
}

template <int PN, typename Real>
hipError_t full_all_r(int mode, const void *args, int lo, int nblk, int lcap, Sink &s)
{
    StageArgs<Real> a = *static_cast<const StageArgs<Real> *>(args);
    void *kargs[] = {&a, &lo, &lcap};
    const dim3 g((PN - lo + 1) * list_grid(nblk, PN)), b(TEAM * TEAM_ROLES);
    return emit(s,
                mode == MODE_STAGE1 ? reinterpret_cast<const void *>(&k_full_all<PN, Real, MODE_STAGE1>)
                                    : reinterpret_cast<const void *>(&k_full_all<PN, Real, MODE_STAGE2>),
                g, b, kargs);
}

hipError_t launch_full_all(int lo, int pn, bool fp32, int mode, const void *args, int nblk, int lcap, Sink &k)
{
    if (nblk <= 0) return hipSuccess;
    if (lo < 0 || lo > pn || pn < 1 || pn > 3 || (mode != MODE_STAGE1 && mode != MODE_STAGE2))
        return hipErrorInvalidValue;
    switch (pn) {
    case 1: return fp32 ? full_all_r<1, float>(mode, args, lo, nblk, lcap, k) : full_all_r<1, double>(mode, args, lo, nblk, lcap, k);
    case 2: return fp32 ? full_all_r<2, float>(mode, args, lo, nblk, lcap, k) : full_all_r<2, double>(mode, args, lo, nblk, lcap, k);
    case 3: return fp32 ? full_all_r<3, float>(mode, args, lo, nblk, lcap, k) : full_all_r<3, double>(mode, args, lo, nblk, lcap, k);
    }
    return hipErrorInvalidValue;
}

template <int B, int PN, typename Real>
hipError_t corr_all_r(const void *args, double dt, int nblk, int lcap, Sink &s)
{
    StageArgs<Real> a = *static_cast<const StageArgs<Real> *>(args);
    void *kargs[] = {&a, &dt, &lcap};
    return emit(s, reinterpret_cast<const void *>(&k_corr_all<B, PN, Real>), dim3((PN - B + 1) * list_grid(nblk, PN)),
                dim3(TEAM * TEAM_ROLES), kargs);
}

template <typename Real>
hipError_t corr_all_t(int b, int pn, const void *args, double dt, int nblk, int lcap, Sink &k)
{
    if (b == 0 && pn == 1) return corr_all_r<0, 1, Real>(args, dt, nblk, lcap, k);
    if (b == 0 && pn == 2) return corr_all_r<0, 2, Real>(args, dt, nblk, lcap, k);
    if (b == 0 && pn == 3) return corr_all_r<0, 3, Real>(args, dt, nblk, lcap, k);
    if (b == 1 && pn == 2) return corr_all_r<1, 2, Real>(args, dt, nblk, lcap, k);
    if (b == 1 && pn == 3) return corr_all_r<1, 3, Real>(args, dt, nblk, lcap, k);
    if (b == 2 && pn == 3) return corr_all_r<2, 3, Real>(args, dt, nblk, lcap, k);
    return hipErrorInvalidValue;
}

template <typename Real>
int host_corr_r(int b, int pn, const void *args, double dt, const signed char *order, int e0, int e1, int nthreads)
{
    const StageArgs<Real> &a = *static_cast<const StageArgs<Real> *>(args);
    if (b == 0 && pn == 1) host_corr_t<0, 1, Real>(a, dt, order, e0, e1, nthreads);
    else if (b == 0 && pn == 2) host_corr_t<0, 2, Real>(a, dt, order, e0, e1, nthreads);
    else if (b == 0 && pn == 3) host_corr_t<0, 3, Real>(a, dt, order, e0, e1, nthreads);
    else if (b == 1 && pn == 2) host_corr_t<1, 2, Real>(a, dt, order, e0, e1, nthreads);
    else if (b == 1 && pn == 3) host_corr_t<1, 3, Real>(a, dt, order, e0, e1, nthreads);
    else if (b == 2 && pn == 3) host_corr_t<2, 3, Real>(a, dt, order, e0, e1, nthreads);
    else return -1;
    return 0;
}

int host_corr(int b, int pn, bool fp32, const void *args, double dt, const signed char *order, int e0, int e1,
              int nthreads)
{
    return fp32 ? host_corr_r<float>(b, pn, args, dt, order, e0, e1, nthreads)
                : host_corr_r<double>(b, pn, args, dt, order, e0, e1, nthreads);
}

hipError_t launch_corr_all(int b, int pn, bool fp32, const void *args, double dt, int nblk, int lcap, Sink &k)
{
    if (nblk <= 0) return hipSuccess;
    return fp32 ? corr_all_t<float>(b, pn, args, dt, nblk, lcap, k) : corr_all_t<double>(b, pn, args, dt, nblk, lcap, k);
}

template <int PN, typename Real>
hipError_t epi_all_r(int mode, int KB, const void *args, int lo, int nblk, int lcap, Sink &s)
{
    StageArgs<Real> a = *static_cast<const StageArgs<Real> *>(args);
    void *kargs[] = {&a, &KB, &lo, &lcap};
    const dim3 g((PN - lo + 1) * nblk), b(BLOCK);
    return emit(s,
                mode == MODE_STAGE1 ? reinterpret_cast<const void *>(&k_epi_all<PN, Real, MODE_STAGE1>)
                                    : reinterpret_cast<const void *>(&k_epi_all<PN, Real, MODE_STAGE2>),
                g, b, kargs);
}

hipError_t launch_epi_all(int b, int pn, bool fp32, int mode, const void *args, int nblk, int lcap, Sink &k)
{
    if (nblk <= 0) return hipSuccess;
    if (b < 0 || b > pn || pn < 1 || pn > 3 || (mode != MODE_STAGE1 && mode != MODE_STAGE2))
        return hipErrorInvalidValue;
    const int KB = (b + 1) * (b + 2) / 2;
    switch (pn) {
    case 1: return fp32 ? epi_all_r<1, float>(mode, KB, args, b, nblk, lcap, k) : epi_all_r<1, double>(mode, KB, args, b, nblk, lcap, k);
    case 2: return fp32 ? epi_all_r<2, float>(mode, KB, args, b, nblk, lcap, k) : epi_all_r<2, double>(mode, KB, args, b, nblk, lcap, k);
    case 3: return fp32 ? epi_all_r<3, float>(mode, KB, args, b, nblk, lcap, k) : epi_all_r<3, double>(mode, KB, args, b, nblk, lcap, k);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_usolve(int p, bool fp32, const void *args, hipStream_t s)
{
    return fp32 ? usolve_r<float>(p, args, s) : usolve_r<double>(p, args, s);
}

template <typename Real>
hipError_t depth_limit_r(int pm, const void *args, double h_min, Sink &s)
{
    StageArgs<Real> a = *static_cast<const StageArgs<Real> *>(args);
    void *kargs[] = {&a, &h_min};
    const dim3 g((a.m.ne + BLOCK - 1) / BLOCK), b(BLOCK);
    switch (pm) {
    case 1: return emit(s, reinterpret_cast<const void *>(&k_depth_limit<1, Real>), g, b, kargs);
    case 2: return emit(s, reinterpret_cast<const void *>(&k_depth_limit<2, Real>), g, b, kargs);
    case 3: return emit(s, reinterpret_cast<const void *>(&k_depth_limit<3, Real>), g, b, kargs);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_depth_limit(int pm, bool fp32, const void *args, double h_min, Sink &k)
{
    if (pm < 1) return hipSuccess;   // order 0 has nothing to scale
    return fp32 ? depth_limit_r<float>(pm, args, h_min, k) : depth_limit_r<double>(pm, args, h_min, k);
}

int mass_partials(int ne) { return (ne + BLOCK - 1) / BLOCK; }

namespace {
template <int P, typename Real, int TILE>
hipError_t batch_pt(int mode, const BatchArgs &b, int grid, Sink &s)
{
    BatchArgs a = b;
    void *kargs[] = {&a};
    const void *fn = mode == MODE_STAGE1 ? reinterpret_cast<const void *>(&k_batch_stage<P, Real, MODE_STAGE1, TILE>)
                                         : reinterpret_cast<const void *>(&k_batch_stage<P, Real, MODE_STAGE2, TILE>);
    return emit(s, fn, dim3(grid), dim3(TILE), kargs);
}

template <typename Real, int TILE>
hipError_t batch_t(int p, int mode, const BatchArgs &b, int grid, Sink &s)
{
    switch (p) {
    case 0: return batch_pt<0, Real, TILE>(mode, b, grid, s);
    case 1: return batch_pt<1, Real, TILE>(mode, b, grid, s);
    case 2: return batch_pt<2, Real, TILE>(mode, b, grid, s);
    case 3: return batch_pt<3, Real, TILE>(mode, b, grid, s);
    }
    return hipErrorInvalidValue;
}

template <typename Real>
hipError_t batch_r(int p, int mode, int tile, const BatchArgs &b, int grid, Sink &s)
{
    switch (tile) {
    case 64: return batch_t<Real, 64>(p, mode, b, grid, s);
    case 128: return batch_t<Real, 128>(p, mode, b, grid, s);
    case 256: return batch_t<Real, 256>(p, mode, b, grid, s);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_batch_stage(int p, bool fp32, int mode, int tile, const BatchArgs &b, int grid, Sink &k)
{
    if (grid <= 0) return hipSuccess;
    return fp32 ? batch_r<float>(p, mode, tile, b, grid, k) : batch_r<double>(p, mode, tile, b, grid, k);
}

template <int P, typename Real>
hipError_t batch_sh_p(int mode, const BatchArgs &b, int grid, Sink &k)
{
    BatchArgs a = b;
    void *kargs[] = {&a};
    const void *fn = mode == MODE_STAGE1 ? reinterpret_cast<const void *>(&k_batch_stage_sh<P, Real, MODE_STAGE1>)
                                         : reinterpret_cast<const void *>(&k_batch_stage_sh<P, Real, MODE_STAGE2>);
    return emit(k, fn, dim3(grid), dim3(BLOCK), kargs);
}

hipError_t launch_batch_stage_sh(int p, bool fp32, int mode, const BatchArgs &b, int grid, Sink &k)
{
    if (grid <= 0) return hipSuccess;
    if (mode != MODE_STAGE1 && mode != MODE_STAGE2) return hipErrorInvalidValue;
    if (fp32 && p == 1) return batch_sh_p<1, float>(mode, b, grid, k);
    if (fp32 && p == 2) return batch_sh_p<2, float>(mode, b, grid, k);
    if (fp32 && p == 3) return batch_sh_p<3, float>(mode, b, grid, k);
    if (!fp32 && p == 1) return batch_sh_p<1, double>(mode, b, grid, k);
    if (!fp32 && p == 2) return batch_sh_p<2, double>(mode, b, grid, k);
    if (!fp32 && p == 3) return batch_sh_p<3, double>(mode, b, grid, k);
    return hipErrorInvalidValue;
}

hipError_t launch_place_items(const unsigned *items, const int *item_off, int nblk, const PoolView &pool, int first,
                              hipStream_t s)
{
    if (nblk <= 0) return hipSuccess;
    if (first % BLOCK != 0 || !pool.items || !pool.nitems) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_place_items, dim3(nblk), dim3(BLOCK), 0, s, items, item_off, pool, first);
    return hipGetLastError();
}

hipError_t launch_batch_clock(InstDesc *inst, const int *flags, int n, Sink &k)
{
    if (n <= 0) return hipSuccess;
    void *kargs[] = {&inst, &flags, &n};
    return emit(k, reinterpret_cast<const void *>(&k_batch_clock), dim3((n + BLOCK - 1) / BLOCK), dim3(BLOCK), kargs);
}

hipError_t launch_relocate(const int *ev, const int *nb, const unsigned char *nbk, const signed char *ep, int ne,
                           int stride, const PoolView &pool, int first, int vbase, hipStream_t s)
{
    if (ne <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_relocate, dim3((ne + BLOCK - 1) / BLOCK), dim3(BLOCK), 0, s, ev, nb, nbk, ep, ne, stride,
                       pool, first, vbase);
    return hipGetLastError();
}

hipError_t launch_batch_indicator(bool fp32, const BatchArgs &b, int grid, Sink &k)
{
    if (grid <= 0) return hipSuccess;
    BatchArgs a = b;
    void *kargs[] = {&a};
    return emit(k, fp32 ? reinterpret_cast<const void *>(&k_batch_indicator<float>)
                        : reinterpret_cast<const void *>(&k_batch_indicator<double>),
                dim3(grid), dim3(BLOCK), kargs);
}

hipError_t launch_batch_apply(int pm, bool fp32, const BatchArgs &b, int grid, Sink &k)
{
    if (grid <= 0) return hipSuccess;
    BatchArgs a = b;
    void *kargs[] = {&a};
    const void *fn = nullptr;
    switch (pm) {
    case 1: fn = fp32 ? reinterpret_cast<const void *>(&k_batch_apply<1, float>)
                      : reinterpret_cast<const void *>(&k_batch_apply<1, double>); break;
    case 2: fn = fp32 ? reinterpret_cast<const void *>(&k_batch_apply<2, float>)
                      : reinterpret_cast<const void *>(&k_batch_apply<2, double>); break;
    case 3: fn = fp32 ? reinterpret_cast<const void *>(&k_batch_apply<3, float>)
                      : reinterpret_cast<const void *>(&k_batch_apply<3, double>); break;
    default: return hipErrorInvalidValue;
    }
    return emit(k, fn, dim3(grid), dim3(BLOCK), kargs);
}

template <typename Real>
hipError_t indicator_r(const void *args, double tau, int p_lo, int p_hi, double *I_out, signed char *p_new,
                       Sink &s)
{
    StageArgs<Real> a = *static_cast<const StageArgs<Real> *>(args);
    void *kargs[] = {&a, &tau, &p_lo, &p_hi, &I_out, &p_new};
    return emit(s, reinterpret_cast<const void *>(&k_indicator<Real>), dim3((a.m.ne + BLOCK - 1) / BLOCK),
                dim3(BLOCK), kargs);
}

hipError_t launch_indicator(bool fp32, const void *args, double tau, int p_lo, int p_hi, double *I_out,
                            signed char *p_new, Sink &k)
{
    return fp32 ? indicator_r<float>(args, tau, p_lo, p_hi, I_out, p_new, k)
                : indicator_r<double>(args, tau, p_lo, p_hi, I_out, p_new, k);
}

hipError_t launch_indicator(bool fp32, const void *args, double tau, int p_lo, int p_hi, double *I_out,
                            signed char *p_new, hipStream_t s)
{
    Sink k;
    k.s = s;
    return launch_indicator(fp32, args, tau, p_lo, p_hi, I_out, p_new, k);
}

template <typename Real>
hipError_t apply_r(int pm, const void *args, const signed char *p_new, signed char *p_cur, int p_base, int lcap,
                   InstDesc *clock, const int *flag, Sink &s)
{
    StageArgs<Real> a = *static_cast<const StageArgs<Real> *>(args);
    void *kargs[] = {&a, &p_new, &p_cur, &p_base, &lcap, &clock, &flag};
    const dim3 g((a.m.ne + BLOCK - 1) / BLOCK), b(BLOCK);
    switch (pm) {
    case 0: return emit(s, reinterpret_cast<const void *>(&k_apply_order<0, Real>), g, b, kargs);
    case 1: return emit(s, reinterpret_cast<const void *>(&k_apply_order<1, Real>), g, b, kargs);
    case 2: return emit(s, reinterpret_cast<const void *>(&k_apply_order<2, Real>), g, b, kargs);
    case 3: return emit(s, reinterpret_cast<const void *>(&k_apply_order<3, Real>), g, b, kargs);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_apply_order(int pm, bool fp32, const void *args, const signed char *p_new, signed char *p_cur,
                              int p_base, int lcap, InstDesc *clock, const int *flag, Sink &k)
{
    return fp32 ? apply_r<float>(pm, args, p_new, p_cur, p_base, lcap, clock, flag, k)
                : apply_r<double>(pm, args, p_new, p_cur, p_base, lcap, clock, flag, k);
}

__global__ void k_inst_set(InstDesc *inst, InstDesc v)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) *inst = v;
}

hipError_t launch_inst_set(InstDesc *inst, const InstDesc &v, hipStream_t s)
{
    hipLaunchKernelGGL(k_inst_set, dim3(1), dim3(64), 0, s, inst, v);
    return hipGetLastError();
}

// Partial sums of the mass reduction for callers that cannot allocate: a
// fixed array on each device (the library holds it until the process ends),
// enough for MASS_SCRATCH_PARTIALS blocks of 256 elements.  Host code never
// passes the array's name to a kernel (on the host it only stands in for the
// symbol): it takes the device address once per device with that device
// current and uses that.
static __device__ __align__(256) double scratch[MASS_SCRATCH_PARTIALS];

namespace {
constexpr int MAX_DEVICES = 64;
std::mutex scratch_mutex;
double *scratch_ptr[MAX_DEVICES] = {};
}  // namespace

hipError_t mass_scratch(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        scratch_ptr[dev] = static_cast<double *>(ptr);
    }
    if (out) *out = scratch_ptr[dev];
    return hipSuccess;
}

hipError_t launch_mass_noalloc(const MeshView &m, bool fp32, const void *C, double *out, hipStream_t s)
{
    const int nb = mass_partials(m.ne);
    if (nb <= 0 || nb > MASS_SCRATCH_PARTIALS) return hipErrorInvalidValue;
    double *part = nullptr;
    hipError_t e = mass_scratch(&part);
    if (e != hipSuccess) return e;
    // every partial the final pass reads is written by the first pass: nothing to clear
    if (fp32)
        hipLaunchKernelGGL(k_mass_partial<float>, dim3(nb), dim3(BLOCK), 0, s, m, static_cast<const float *>(C), part);
    else
        hipLaunchKernelGGL(k_mass_partial<double>, dim3(nb), dim3(BLOCK), 0, s, m, static_cast<const double *>(C),
                           part);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(BLOCK), 0, s, part, nb, out);
    return hipGetLastError();
}

hipError_t launch_mass(const MeshView &m, bool fp32, const void *C, double *partial, double *out,
                       hipStream_t s)
{
    const int nb = mass_partials(m.ne);
    if (nb <= 0) return hipErrorInvalidValue;
    if (fp32)
        hipLaunchKernelGGL(k_mass_partial<float>, dim3(nb), dim3(BLOCK), 0, s, m,
                           static_cast<const float *>(C), partial);
    else
        hipLaunchKernelGGL(k_mass_partial<double>, dim3(nb), dim3(BLOCK), 0, s, m,
                           static_cast<const double *>(C), partial);
    hipLaunchKernelGGL(k_mass_final, dim3(1), dim3(BLOCK), 0, s, partial, nb, out);
    return hipGetLastError();
}

}  // namespace swe
