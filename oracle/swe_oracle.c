/*
 * Oracle for the quadrature-free DG discretisation of the 2D shallow water
 * equations (Faghih-Naini et al., "p-adaptive discontinuous Galerkin method for
 * the shallow water equations on heterogeneous computing architectures").
 *
 * TEST INFRASTRUCTURE ONLY.  It is linked by the test-suite, by the package's
 * smoke check and by the CPU-baseline leg of the benchmark; the product library
 * never links, loads or calls it, and it shares no code, header or table with
 * the HIP path.
 *
 * What it computes, in plain FP64, element by element and edge by edge:
 *   - the compact system c = (xi, U, V), flux A(c,u) and source r(c,u) of
 *     eqs. (compact_qf_1), (compact_qf_2), (def_A_h_qf);
 *   - the semi-discrete form (variational_disc_1): volume term (A, grad phi),
 *     source term (r, phi) and edge term <A_hat, phi> with the Lax-Friedrichs
 *     flux and the penalty lambda of eq. (eq:lambda) taken from constant parts
 *     (Sec. "Algorithmic adaptation: order separation");
 *   - the auxiliary system u H = q (variational_disc_2) with the truncated
 *     depth expansion K(p,i,j) of Sec. "order separation", solved by LU with
 *     partial pivoting;
 *   - two-stage SSP Runge-Kutta in Shu-Osher form (Sec. "Quadrature-free DG
 *     formulation", time discretisation);
 *   - optionally, a minimum depth control after every stage (the paper lists
 *     such a kernel among those of its code, Sec. "Performance results",
 *     without defining it; the reading is stated at depth_limit_elem).
 * The method integrates products of polynomials exactly with precomputed
 * basis-product integrals.  The oracle instead evaluates every integral by
 * Gaussian quadrature that is exact for the polynomial degree of its
 * integrand, so both compute the same numbers by different algorithms.
 *
 * Readings of points the paper leaves open (each also listed in the design
 * notes): basis = Gram-Schmidt of the monomials 1,x,y,x^2,xy,y^2,x^3,... on the
 * reference triangle with positive leading coefficient; bathymetry continuous
 * and piecewise linear from vertex depths; K(p,i,j) = K(max(deg i, deg j));
 * land ghost state = mirror of q and u with zero mass flux; open sea ghost
 * xi = xi_hat(t), q and u copied; lambda from element means of xi and u plus
 * the bathymetry at the edge midpoint; linear friction read as -kappa*q;
 * quadratic friction -C_f |u_mean| u.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define KMAX 10
#define NCON_MAX 16

static const int K_OF_P[4] = {1, 3, 6, 10};
/* polynomial degree of basis function i (hierarchical ordering) */
static const int DEG_OF[KMAX] = {0, 1, 1, 2, 2, 2, 3, 3, 3, 3};
/* monomial exponents in Gram-Schmidt order */
static const int MONO_A[KMAX] = {0, 1, 0, 2, 1, 0, 3, 2, 1, 0};
static const int MONO_B[KMAX] = {0, 0, 1, 0, 1, 2, 0, 1, 2, 3};

/* ------------------------------------------------------------------ */
/* Gauss-Legendre rule on [0,1] by Newton iteration on P_n.            */
/* ------------------------------------------------------------------ */
static void gauss_legendre01(int n, long double *t, long double *w)
{
    for (int i = 0; i < n; ++i) {
        long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (n + 0.5L));
        long double p0 = 1, p1 = z, dp = 1;
        for (int it = 0; it < 200; ++it) {
            p0 = 1.0L;
            p1 = z;
            for (int k = 2; k <= n; ++k) {
                long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) { p1 = z; p0 = 1.0L; }
            dp = n * (z * p1 - p0) / (z * z - 1.0L);
            long double dz = p1 / dp;
            z -= dz;
            if (fabsl(dz) < 1e-21L) break;
        }
        p0 = 1.0L;
        p1 = z;
        for (int k = 2; k <= n; ++k) {
            long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0L);
        t[i] = 0.5L * (z + 1.0L);
        w[i] = 1.0L / ((1.0L - z * z) * dp * dp);  /* 2/((1-z^2)P'^2) halved for [0,1] */
    }
}

/* Collapsed (Duffy) product rule on the reference triangle
 * {x,y >= 0, x + y <= 1}: x = a, y = b (1 - a), weight w_a w_b (1 - a).
 * With n points per direction it integrates total degree 2n-2 exactly. */
typedef struct {
    int n;                       /* number of points */
    double x[256], y[256], w[256];
} tri_rule;

static void make_tri_rule(int n1, tri_rule *r)
{
    long double t[16], w[16];
    gauss_legendre01(n1, t, w);
    r->n = 0;
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            r->x[r->n] = (double)t[i];
            r->y[r->n] = (double)(t[j] * (1.0L - t[i]));
            r->w[r->n] = (double)(w[i] * w[j] * (1.0L - t[i]));
            r->n++;
        }
}

/* ------------------------------------------------------------------ */
/* Hierarchical orthonormal basis on the reference triangle, built by  */
/* Gram-Schmidt (twice, in long double) of centred monomials.  Centring */
/* at (1/3,1/3) only improves conditioning: within the degree-graded    */
/* order it leaves every partial span, hence the basis, unchanged.      */
/* ------------------------------------------------------------------ */
static double BASIS_A[KMAX][KMAX];   /* phi_i = sum_m A[i][m] (x-1/3)^a_m (y-1/3)^b_m */
static int basis_ready = 0;

static long double powl_i(long double x, int k)
{
    long double r = 1.0L;
    for (int i = 0; i < k; ++i) r *= x;
    return r;
}

static void build_basis(void)
{
    if (basis_ready) return;
    long double t[16], w[16];
    const int n1 = 8;  /* exact to degree 14 >= 6 */
    gauss_legendre01(n1, t, w);
    long double px[64], py[64], pw[64];
    int np = 0;
    for (int i = 0; i < n1; ++i)
        for (int j = 0; j < n1; ++j) {
            px[np] = t[i];
            py[np] = t[j] * (1.0L - t[i]);
            pw[np] = w[i] * w[j] * (1.0L - t[i]);
            np++;
        }
    long double M[64][KMAX];  /* centred monomial values */
    for (int q = 0; q < np; ++q)
        for (int m = 0; m < KMAX; ++m)
            M[q][m] = powl_i(px[q] - 1.0L / 3.0L, MONO_A[m]) * powl_i(py[q] - 1.0L / 3.0L, MONO_B[m]);
    long double A[KMAX][KMAX];
    memset(A, 0, sizeof(A));
    for (int i = 0; i < KMAX; ++i) {
        long double v[KMAX] = {0};
        v[i] = 1.0L;
        for (int pass = 0; pass < 2; ++pass) {
            for (int j = 0; j < i; ++j) {
                long double ip = 0.0L;
                for (int q = 0; q < np; ++q) {
                    long double a = 0.0L, b = 0.0L;
                    for (int m = 0; m < KMAX; ++m) {
                        a += v[m] * M[q][m];
                        b += A[j][m] * M[q][m];
                    }
                    ip += pw[q] * a * b;
                }
                for (int m = 0; m < KMAX; ++m) v[m] -= ip * A[j][m];
            }
        }
        long double nn = 0.0L;
        for (int q = 0; q < np; ++q) {
            long double a = 0.0L;
            for (int m = 0; m < KMAX; ++m) a += v[m] * M[q][m];
            nn += pw[q] * a * a;
        }
        long double s = 1.0L / sqrtl(nn);
        for (int m = 0; m < KMAX; ++m) A[i][m] = v[m] * s;
    }
    for (int i = 0; i < KMAX; ++i)
        for (int m = 0; m < KMAX; ++m) BASIS_A[i][m] = (double)A[i][m];
    basis_ready = 1;
}

/* Values and reference gradients of the first K basis functions at (x,y). */
static void basis_eval(int K, double x, double y, double *phi, double *dx, double *dy)
{
    double X = x - 1.0 / 3.0, Y = y - 1.0 / 3.0;
    double Xp[4] = {1.0, X, X * X, X * X * X};
    double Yp[4] = {1.0, Y, Y * Y, Y * Y * Y};
    double mv[KMAX], mx[KMAX], my[KMAX];
    for (int m = 0; m < KMAX; ++m) {
        int a = MONO_A[m], b = MONO_B[m];
        mv[m] = Xp[a] * Yp[b];
        mx[m] = a > 0 ? a * Xp[a - 1] * Yp[b] : 0.0;
        my[m] = b > 0 ? b * Xp[a] * Yp[b - 1] : 0.0;
    }
    for (int i = 0; i < K; ++i) {
        double v = 0.0, gx = 0.0, gy = 0.0;
        for (int m = 0; m < KMAX; ++m) {
            v += BASIS_A[i][m] * mv[m];
            gx += BASIS_A[i][m] * mx[m];
            gy += BASIS_A[i][m] * my[m];
        }
        phi[i] = v;
        if (dx) dx[i] = gx;
        if (dy) dy[i] = gy;
    }
}

/* ------------------------------------------------------------------ */
/* Oracle state                                                        */
/* ------------------------------------------------------------------ */
typedef struct {
    int nv, ne, pmax, K;
    double *vx, *vy, *hb;
    int *tri;       /* [ne][3] */
    int *nb;        /* [ne][3] neighbour element or -1 */
    int *btype;     /* [ne][3] -1 interior, 0 land, 1 open */
    int *p;         /* [ne] */
    double *Bi;     /* [ne][4] inverse Jacobian, row-major (Bi[0]=d xhat/dx ...) */
    double *det;    /* [ne] |det B| = 2*area */
    /* physics */
    double g, fc, fric_coef;
    int friction;
    int ncon;
    double amp[NCON_MAX], omega[NCON_MAX], phase[NCON_MAX];
    double *src;    /* optional [ne][3][K] */
    int exact_H;    /* diagnostics: use the untruncated depth in u H = q */
    double h_min;   /* minimum depth control after every stage (0: off) */
    /* scratch */
    double *u;      /* [ne][2][K] */
    tri_rule el_rule;
    int n_edge;
    double et[32], ew[32];
} orc;

static double xi_hat(const orc *o, double t)
{
    double s = 0.0;
    for (int i = 0; i < o->ncon; ++i) s += o->amp[i] * sin(o->omega[i] * t + o->phase[i]);
    return s;
}

typedef struct { int lo, hi, e, k; } edge_key;

static int cmp_edge(const void *a, const void *b)
{
    const edge_key *x = (const edge_key *)a, *y = (const edge_key *)b;
    if (x->lo != y->lo) return x->lo < y->lo ? -1 : 1;
    if (x->hi != y->hi) return x->hi < y->hi ? -1 : 1;
    if (x->e != y->e) return x->e < y->e ? -1 : 1;
    return x->k - y->k;
}

static void set_rules(orc *o)
{
    /* element integrands have degree <= 3p (u-solve), edge integrands <= 3p */
    int p = o->pmax;
    make_tri_rule((3 * p + 2) / 2 + 1, &o->el_rule);
    long double t[32], w[32];
    o->n_edge = (3 * p + 1) / 2 + 1;
    gauss_legendre01(o->n_edge, t, w);
    for (int i = 0; i < o->n_edge; ++i) {
        o->et[i] = (double)t[i];
        o->ew[i] = (double)w[i];
    }
}

void orc_destroy(void *h)
{
    orc *o = (orc *)h;
    if (!o) return;
    free(o->vx); free(o->vy); free(o->hb); free(o->tri); free(o->nb); free(o->btype);
    free(o->p); free(o->Bi); free(o->det); free(o->src); free(o->u);
    free(o);
}

/* tag[e*3+k]: -1 interior/auto, 0 land, 1 open.  Returns NULL on an invalid
 * mesh (non-positive area, an edge shared by more than two elements). */
void *orc_create(int nv, const double *vxy, const double *hb, int ne, const int *tri,
                 const signed char *tag, int pmax)
{
    if (nv <= 0 || ne <= 0 || pmax < 0 || pmax > 3) return NULL;
    build_basis();
    orc *o = (orc *)calloc(1, sizeof(orc));
    o->nv = nv; o->ne = ne; o->pmax = pmax; o->K = K_OF_P[pmax];
    o->vx = malloc(sizeof(double) * nv); o->vy = malloc(sizeof(double) * nv);
    o->hb = malloc(sizeof(double) * nv);
    for (int v = 0; v < nv; ++v) { o->vx[v] = vxy[2 * v]; o->vy[v] = vxy[2 * v + 1]; o->hb[v] = hb[v]; }
    o->tri = malloc(sizeof(int) * 3 * ne); memcpy(o->tri, tri, sizeof(int) * 3 * ne);
    o->nb = malloc(sizeof(int) * 3 * ne); o->btype = malloc(sizeof(int) * 3 * ne);
    o->p = malloc(sizeof(int) * ne);
    o->Bi = malloc(sizeof(double) * 4 * ne); o->det = malloc(sizeof(double) * ne);
    o->u = calloc((size_t)ne * 2 * o->K, sizeof(double));
    o->g = 9.81;
    for (int e = 0; e < ne; ++e) {
        o->p[e] = pmax;
        int a = tri[3 * e], b = tri[3 * e + 1], c = tri[3 * e + 2];
        if (a < 0 || b < 0 || c < 0 || a >= nv || b >= nv || c >= nv) { orc_destroy(o); return NULL; }
        double b00 = o->vx[b] - o->vx[a], b01 = o->vx[c] - o->vx[a];
        double b10 = o->vy[b] - o->vy[a], b11 = o->vy[c] - o->vy[a];
        double d = b00 * b11 - b01 * b10;
        if (!(d > 0.0)) { orc_destroy(o); return NULL; }
        o->det[e] = d;
        o->Bi[4 * e + 0] = b11 / d;  o->Bi[4 * e + 1] = -b01 / d;
        o->Bi[4 * e + 2] = -b10 / d; o->Bi[4 * e + 3] = b00 / d;
    }
    edge_key *ek = malloc(sizeof(edge_key) * 3 * (size_t)ne);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            int va = tri[3 * e + (k + 1) % 3], vb = tri[3 * e + (k + 2) % 3];
            edge_key x = {va < vb ? va : vb, va < vb ? vb : va, e, k};
            ek[3 * e + k] = x;
            o->nb[3 * e + k] = -1;
        }
    qsort(ek, 3 * (size_t)ne, sizeof(edge_key), cmp_edge);
    size_t i = 0, n3 = 3 * (size_t)ne;
    while (i < n3) {
        size_t j = i + 1;
        while (j < n3 && ek[j].lo == ek[i].lo && ek[j].hi == ek[i].hi) ++j;
        if (j - i > 2) { free(ek); orc_destroy(o); return NULL; }
        if (j - i == 2) {
            o->nb[3 * ek[i].e + ek[i].k] = ek[i + 1].e;
            o->nb[3 * ek[i + 1].e + ek[i + 1].k] = ek[i].e;
        }
        i = j;
    }
    free(ek);
    for (int e = 0; e < ne; ++e)
        for (int k = 0; k < 3; ++k) {
            if (o->nb[3 * e + k] >= 0) o->btype[3 * e + k] = -1;
            else o->btype[3 * e + k] = (tag && tag[3 * e + k] == 1) ? 1 : 0;
        }
    set_rules(o);
    return o;
}

int orc_set_physics(void *h, double g, double fc, int friction, double coef)
{
    orc *o = (orc *)h;
    if (friction < 0 || friction > 2 || !(g > 0.0)) return -1;
    o->g = g; o->fc = fc; o->friction = friction; o->fric_coef = coef;
    return 0;
}

int orc_set_open(void *h, int ncon, const double *amp, const double *omega, const double *phase)
{
    orc *o = (orc *)h;
    if (ncon < 0 || ncon > NCON_MAX) return -1;
    o->ncon = ncon;
    for (int i = 0; i < ncon; ++i) { o->amp[i] = amp[i]; o->omega[i] = omega[i]; o->phase[i] = phase[i]; }
    return 0;
}

int orc_set_order(void *h, const int *p)
{
    orc *o = (orc *)h;
    for (int e = 0; e < o->ne; ++e) if (p[e] < 0 || p[e] > o->pmax) return -1;
    memcpy(o->p, p, sizeof(int) * o->ne);
    return 0;
}

int orc_get_order(void *h, int *p)
{
    orc *o = (orc *)h;
    memcpy(p, o->p, sizeof(int) * o->ne);
    return 0;
}

int orc_set_source(void *h, const double *src)
{
    orc *o = (orc *)h;
    free(o->src);
    o->src = NULL;
    if (src) {
        size_t n = (size_t)o->ne * 3 * o->K;
        o->src = malloc(sizeof(double) * n);
        memcpy(o->src, src, sizeof(double) * n);
    }
    return 0;
}

void orc_set_exact_H(void *h, int on) { ((orc *)h)->exact_H = on; }

/* reference coordinates of physical point (x,y) in element e */
static void to_ref(const orc *o, int e, double x, double y, double *xh, double *yh)
{
    int a = o->tri[3 * e];
    double dx = x - o->vx[a], dy = y - o->vy[a];
    const double *B = o->Bi + 4 * e;
    *xh = B[0] * dx + B[1] * dy;
    *yh = B[2] * dx + B[3] * dy;
}

/* bathymetry (linear interpolation of vertex depths) at reference point */
static double hb_at(const orc *o, int e, double xh, double yh)
{
    const int *t = o->tri + 3 * e;
    return o->hb[t[0]] * (1.0 - xh - yh) + o->hb[t[1]] * xh + o->hb[t[2]] * yh;
}

/* ------------------------------------------------------------------ */
/* u H = q: H_ij = int (sum_{n<=K(max deg)} xi_n phi_n + h_b) phi_i phi_j */
/* ------------------------------------------------------------------ */
static int lu_solve(int n, double *A, double *b1, double *b2)
{
    int piv[KMAX];
    for (int k = 0; k < n; ++k) {
        int r = k;
        double best = fabs(A[k * n + k]);
        for (int i = k + 1; i < n; ++i)
            if (fabs(A[i * n + k]) > best) { best = fabs(A[i * n + k]); r = i; }
        if (!(best > 0.0)) return -1;
        piv[k] = r;
        if (r != k) {
            for (int j = 0; j < n; ++j) { double tmp = A[k * n + j]; A[k * n + j] = A[r * n + j]; A[r * n + j] = tmp; }
            double t1 = b1[k]; b1[k] = b1[r]; b1[r] = t1;
            double t2 = b2[k]; b2[k] = b2[r]; b2[r] = t2;
        }
        for (int i = k + 1; i < n; ++i) {
            double f = A[i * n + k] / A[k * n + k];
            A[i * n + k] = f;
            for (int j = k + 1; j < n; ++j) A[i * n + j] -= f * A[k * n + j];
            b1[i] -= f * b1[k];
            b2[i] -= f * b2[k];
        }
    }
    (void)piv;
    for (int i = n - 1; i >= 0; --i) {
        for (int j = i + 1; j < n; ++j) { b1[i] -= A[i * n + j] * b1[j]; b2[i] -= A[i * n + j] * b2[j]; }
        b1[i] /= A[i * n + i];
        b2[i] /= A[i * n + i];
    }
    return 0;
}

static int usolve_elem(const orc *o, int e, const double *c, double *u)
{
    const int K = o->K, Ke = K_OF_P[o->p[e]];
    const double *ce = c + (size_t)e * 3 * K;
    const double s = sqrt(o->det[e]);
    double H[KMAX * KMAX], bu[KMAX], bv[KMAX];
    memset(H, 0, sizeof(H));
    memset(bu, 0, sizeof(bu));
    memset(bv, 0, sizeof(bv));
    const tri_rule *R = &o->el_rule;
    for (int q = 0; q < R->n; ++q) {
        double phi[KMAX];
        basis_eval(Ke, R->x[q], R->y[q], phi, NULL, NULL);
        double hb = hb_at(o, e, R->x[q], R->y[q]);
        /* depth truncated to the first K(d) modes, d = 0..3 */
        double xi_tr[4];
        for (int d = 0; d < 4; ++d) {
            double acc = 0.0;
            int kd = K_OF_P[d] < Ke ? K_OF_P[d] : Ke;
            for (int n = 0; n < kd; ++n) acc += ce[n] * phi[n];
            xi_tr[d] = acc / s;
        }
        double Uv = 0.0, Vv = 0.0;
        for (int n = 0; n < Ke; ++n) { Uv += ce[K + n] * phi[n]; Vv += ce[2 * K + n] * phi[n]; }
        Uv /= s;
        Vv /= s;
        double w = R->w[q] * o->det[e];
        for (int i = 0; i < Ke; ++i) {
            for (int j = 0; j < Ke; ++j) {
                int d = DEG_OF[i] > DEG_OF[j] ? DEG_OF[i] : DEG_OF[j];
                if (o->exact_H) d = 3;
                H[i * Ke + j] += w * (xi_tr[d] + hb) * phi[i] * phi[j] / (s * s);
            }
            bu[i] += w * Uv * phi[i] / s;
            bv[i] += w * Vv * phi[i] / s;
        }
    }
    if (lu_solve(Ke, H, bu, bv) != 0) return -1;
    double *ue = u + (size_t)e * 2 * K;
    for (int i = 0; i < K; ++i) {
        ue[i] = i < Ke ? bu[i] : 0.0;
        ue[K + i] = i < Ke ? bv[i] : 0.0;
    }
    return 0;
}

int orc_usolve(void *h, const double *c, double *u)
{
    orc *o = (orc *)h;
    for (int e = 0; e < o->ne; ++e)
        if (usolve_elem(o, e, c, u) != 0) return -4;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Right-hand side L(c,t) = (A, grad phi) + (r, phi) - <A_hat, phi>     */
/* ------------------------------------------------------------------ */
static void flux_normal(double g, double xi, double U, double V, double u, double v, double hb,
                        double nx, double ny, double *F)
{
    double P = 0.5 * g * xi * (xi + 2.0 * hb);
    F[0] = U * nx + V * ny;
    F[1] = (U * u + P) * nx + U * v * ny;
    F[2] = V * u * nx + (V * v + P) * ny;
}

static void eval_fields(const orc *o, int e, const double *c, const double *u, double xh, double yh,
                        double *phi, double *fc, double *fu)
{
    const int K = o->K, Ke = K_OF_P[o->p[e]];
    basis_eval(Ke, xh, yh, phi, NULL, NULL);
    const double *ce = c + (size_t)e * 3 * K, *ue = u + (size_t)e * 2 * K;
    const double s = sqrt(o->det[e]);
    for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int n = 0; n < Ke; ++n) acc += ce[j * K + n] * phi[n];
        fc[j] = acc / s;
    }
    for (int j = 0; j < 2; ++j) {
        double acc = 0.0;
        for (int n = 0; n < Ke; ++n) acc += ue[j * K + n] * phi[n];
        fu[j] = acc / s;
    }
}

static void rhs_volume(const orc *o, int e, const double *c, const double *u, double *L)
{
    const int K = o->K, Ke = K_OF_P[o->p[e]];
    const double s = sqrt(o->det[e]);
    const double area = 0.5 * o->det[e];
    const double *B = o->Bi + 4 * e;
    const int *t = o->tri + 3 * e;
    const double dhx = B[0] * (o->hb[t[1]] - o->hb[t[0]]) + B[2] * (o->hb[t[2]] - o->hb[t[0]]);
    const double dhy = B[1] * (o->hb[t[1]] - o->hb[t[0]]) + B[3] * (o->hb[t[2]] - o->hb[t[0]]);
    const double *ue = u + (size_t)e * 2 * K;
    /* constant part of the velocity: u_1 phi_1 with phi_1 = 1/sqrt(area) */
    const double ub = ue[0] / sqrt(area), vb = ue[K] / sqrt(area);
    double tau = 0.0;
    if (o->friction == 2) tau = o->fric_coef * sqrt(ub * ub + vb * vb);
    double *Le = L + (size_t)e * 3 * K;
    const tri_rule *R = &o->el_rule;
    for (int q = 0; q < R->n; ++q) {
        double phi[KMAX], dpx[KMAX], dpy[KMAX], fc[3], fu[2];
        basis_eval(Ke, R->x[q], R->y[q], phi, dpx, dpy);
        eval_fields(o, e, c, u, R->x[q], R->y[q], phi, fc, fu);
        double hb = hb_at(o, e, R->x[q], R->y[q]);
        double xi = fc[0], U = fc[1], V = fc[2], uu = fu[0], vv = fu[1];
        double P = 0.5 * o->g * xi * (xi + 2.0 * hb);
        double A[3][2] = {{U, V}, {U * uu + P, U * vv}, {V * uu, V * vv + P}};
        double r[3];
        r[0] = 0.0;
        r[1] = o->fc * V + o->g * xi * dhx;
        r[2] = -o->fc * U + o->g * xi * dhy;
        if (o->friction == 1) { r[1] -= o->fric_coef * U; r[2] -= o->fric_coef * V; }
        if (o->friction == 2) { r[1] -= tau * uu; r[2] -= tau * vv; }
        double w = R->w[q] * o->det[e];
        for (int i = 0; i < Ke; ++i) {
            /* physical gradient of phi_i = B^{-T} grad_ref / s */
            double gx = (B[0] * dpx[i] + B[2] * dpy[i]) / s;
            double gy = (B[1] * dpx[i] + B[3] * dpy[i]) / s;
            for (int j = 0; j < 3; ++j)
                Le[j * K + i] += w * (A[j][0] * gx + A[j][1] * gy + r[j] * phi[i] / s);
        }
    }
}

static void rhs_edges(const orc *o, double t, const double *c, const double *u, double *L)
{
    const int K = o->K;
    const double g = o->g;
    const double xh_t = xi_hat(o, t);
    for (int e = 0; e < o->ne; ++e) {
        for (int k = 0; k < 3; ++k) {
            int nb = o->nb[3 * e + k];
            if (nb >= 0 && nb < e) continue;  /* each interior edge once */
            int bt = o->btype[3 * e + k];
            int va = o->tri[3 * e + (k + 1) % 3], vb = o->tri[3 * e + (k + 2) % 3];
            double dx = o->vx[vb] - o->vx[va], dy = o->vy[vb] - o->vy[va];
            double len = sqrt(dx * dx + dy * dy);
            double nx = dy / len, ny = -dx / len;
            double hmid = 0.5 * (o->hb[va] + o->hb[vb]);
            double am = 0.5 * o->det[e];
            double ubm = u[(size_t)e * 2 * K] / sqrt(am), vbm = u[(size_t)e * 2 * K + K] / sqrt(am);
            double xbm = c[(size_t)e * 3 * K] / sqrt(am);
            double unm = fabs(ubm * nx + vbm * ny), unp, xbp;
            if (nb >= 0) {
                double ap = 0.5 * o->det[nb];
                double ubp = u[(size_t)nb * 2 * K] / sqrt(ap), vbp = u[(size_t)nb * 2 * K + K] / sqrt(ap);
                unp = fabs(ubp * nx + vbp * ny);
                xbp = c[(size_t)nb * 3 * K] / sqrt(ap);
            } else if (bt == 0) {
                unp = unm;          /* mirrored velocity has the opposite normal part */
                xbp = xbm;
            } else {
                unp = unm;
                xbp = xh_t;
            }
            double lam = fmax(unm, unp) + fmax(sqrt(g * (xbm + hmid)), sqrt(g * (xbp + hmid)));
            const int Km = K_OF_P[o->p[e]];
            const int Kp = nb >= 0 ? K_OF_P[o->p[nb]] : 0;
            const double sm = sqrt(o->det[e]), sp = nb >= 0 ? sqrt(o->det[nb]) : 1.0;
            double *Lm = L + (size_t)e * 3 * K;
            double *Lp = nb >= 0 ? L + (size_t)nb * 3 * K : NULL;
            for (int gq = 0; gq < o->n_edge; ++gq) {
                double tt = o->et[gq], wq = o->ew[gq] * len;
                double X = o->vx[va] + tt * dx, Y = o->vy[va] + tt * dy;
                double hb = o->hb[va] * (1.0 - tt) + o->hb[vb] * tt;
                double xh, yh, phim[KMAX], phip[KMAX], cm[3], um[2], cp[3], up[2];
                to_ref(o, e, X, Y, &xh, &yh);
                eval_fields(o, e, c, u, xh, yh, phim, cm, um);
                if (nb >= 0) {
                    to_ref(o, nb, X, Y, &xh, &yh);
                    eval_fields(o, nb, c, u, xh, yh, phip, cp, up);
                } else if (bt == 0) {
                    double qn = cm[1] * nx + cm[2] * ny, qt = -cm[1] * ny + cm[2] * nx;
                    double vn = um[0] * nx + um[1] * ny, vt = -um[0] * ny + um[1] * nx;
                    cp[0] = cm[0];
                    cp[1] = -qn * nx - qt * ny;
                    cp[2] = -qn * ny + qt * nx;
                    up[0] = -vn * nx - vt * ny;
                    up[1] = -vn * ny + vt * nx;
                } else {
                    cp[0] = xh_t; cp[1] = cm[1]; cp[2] = cm[2];
                    up[0] = um[0]; up[1] = um[1];
                }
                double Fm[3], Fp[3], Ah[3];
                flux_normal(g, cm[0], cm[1], cm[2], um[0], um[1], hb, nx, ny, Fm);
                flux_normal(g, cp[0], cp[1], cp[2], up[0], up[1], hb, nx, ny, Fp);
                for (int j = 0; j < 3; ++j) Ah[j] = 0.5 * (Fm[j] + Fp[j] + lam * (cm[j] - cp[j]));
                if (nb < 0 && bt == 0) Ah[0] = 0.0;   /* land: q.n = 0, no mass flux */
                for (int i = 0; i < Km; ++i)
                    for (int j = 0; j < 3; ++j) Lm[j * K + i] -= wq * Ah[j] * phim[i] / sm;
                if (nb >= 0)
                    for (int i = 0; i < Kp; ++i)
                        for (int j = 0; j < 3; ++j) Lp[j * K + i] += wq * Ah[j] * phip[i] / sp;
            }
        }
    }
}

int orc_rhs(void *h, double t, const double *c, double *L)
{
    orc *o = (orc *)h;
    int rc = orc_usolve(h, c, o->u);
    if (rc) return rc;
    size_t n = (size_t)o->ne * 3 * o->K;
    memset(L, 0, sizeof(double) * n);
    for (int e = 0; e < o->ne; ++e) rhs_volume(o, e, c, o->u, L);
    rhs_edges(o, t, c, o->u, L);
    if (o->src)
        for (size_t i = 0; i < n; ++i) L[i] += o->src[i];
    for (int e = 0; e < o->ne; ++e) {
        int Ke = K_OF_P[o->p[e]];
        for (int j = 0; j < 3; ++j)
            for (int i = Ke; i < o->K; ++i) L[(size_t)e * 3 * o->K + j * o->K + i] = 0.0;
    }
    return 0;
}

/* mean depth check: xi_mean + mean h_b > 0 and every coefficient finite */
static int depth_ok(const orc *o, const double *c)
{
    for (int e = 0; e < o->ne; ++e) {
        const int *t = o->tri + 3 * e;
        double a = 0.5 * o->det[e];
        double H = c[(size_t)e * 3 * o->K] / sqrt(a) + (o->hb[t[0]] + o->hb[t[1]] + o->hb[t[2]]) / 3.0;
        if (!(H > 0.0)) return 0;
        for (int i = 0; i < 3 * o->K; ++i)
            if (!isfinite(c[(size_t)e * 3 * o->K + i])) return 0;
    }
    return 1;
}

/* ------------------------------------------------------------------ */
/* Minimum depth control.  Reading of the paper's "minimum depth control */
/* to avoid negative depths" (a kernel of its code, Sec. "Performance    */
/* results"; not defined there): after every RK stage, an element whose  */
/* total depth H = xi + h_b is below h_min at one of its check points    */
/* (its three vertices and its three edge midpoints) has the deviation   */
/* of H from its element mean scaled by                                  */
/*   theta = (mean H - h_min) / (mean H - min_j H(x_j)),                 */
/* or 0 when mean H <= h_min, which brings H up to h_min at the check    */
/* points and keeps the mean (the mass); the momentum's deviation from   */
/* its mean is scaled by the same theta.  h_b cannot change, so xi takes */
/* the scaled deviation of H minus that of h_b:                          */
/*   xi' = mean xi + theta (xi - mean xi) + (theta - 1)(h_b - mean h_b). */
/* An element of order 0 has no mode to scale and is left alone.         */
/* ------------------------------------------------------------------ */
static int depth_limit_elem(const orc *o, int e, double *ce, double h_min)
{
    const int K = o->K, Ke = K_OF_P[o->p[e]];
    if (Ke < 3) return 0;
    const int *t = o->tri + 3 * e;
    const double sd = sqrt(o->det[e]), area = 0.5 * o->det[e];
    const double hbm = (o->hb[t[0]] + o->hb[t[1]] + o->hb[t[2]]) / 3.0;
    const double Hm = ce[0] / sqrt(area) + hbm;
    static const double px[6] = {0.0, 1.0, 0.0, 0.5, 0.0, 0.5};
    static const double py[6] = {0.0, 0.0, 1.0, 0.5, 0.5, 0.0};
    double Hlow = INFINITY, phi[KMAX];
    for (int j = 0; j < 6; ++j) {
        basis_eval(Ke, px[j], py[j], phi, NULL, NULL);
        double xi = 0.0;
        for (int n = 0; n < Ke; ++n) xi += ce[n] * phi[n];
        const double H = xi / sd + hb_at(o, e, px[j], py[j]);
        if (H < Hlow) Hlow = H;
    }
    if (!(Hlow < h_min)) return 0;
    const double theta = Hm > h_min ? (Hm - h_min) / (Hm - Hlow) : 0.0;
    /* modes of h_b - mean h_b: its L2 projection (h_b is linear, so exact) */
    double bq[3] = {0.0, 0.0, 0.0};
    const tri_rule *R = &o->el_rule;
    for (int q = 0; q < R->n; ++q) {
        basis_eval(3, R->x[q], R->y[q], phi, NULL, NULL);
        const double f = (hb_at(o, e, R->x[q], R->y[q]) - hbm) * R->w[q] * o->det[e] / sd;
        for (int n = 0; n < 3; ++n) bq[n] += f * phi[n];
    }
    for (int n = 1; n < Ke; ++n) {
        ce[n] = theta * ce[n] + (n < 3 ? (theta - 1.0) * bq[n] : 0.0);
        ce[K + n] *= theta;
        ce[2 * K + n] *= theta;
    }
    return 1;
}

/* the control on every element; returns how many were changed */
int orc_depth_limit(void *h, double *c, double h_min)
{
    orc *o = (orc *)h;
    int n = 0;
    for (int e = 0; e < o->ne; ++e) n += depth_limit_elem(o, e, c + (size_t)e * 3 * o->K, h_min);
    return n;
}

int orc_set_depth_limit(void *h, double h_min)
{
    if (!(h_min >= 0.0) || !isfinite(h_min)) return -1;
    ((orc *)h)->h_min = h_min;
    return 0;
}

/* ------------------------------------------------------------------ */
/* p-adaptivity stand-in: jumps of the P1 part of xi at edge midpoints */
/* ------------------------------------------------------------------ */
static double xi_p1_at(const orc *o, int e, const double *c, double x, double y)
{
    double xh, yh, phi[KMAX];
    to_ref(o, e, x, y, &xh, &yh);
    basis_eval(3, xh, yh, phi, NULL, NULL);
    const double *ce = c + (size_t)e * 3 * o->K;
    int Ke = K_OF_P[o->p[e]];
    double acc = 0.0;
    for (int n = 0; n < 3 && n < Ke; ++n) acc += ce[n] * phi[n];
    return acc / sqrt(o->det[e]);
}

int orc_indicator(void *h, double t, const double *c, double *I)
{
    orc *o = (orc *)h;
    double xt = xi_hat(o, t);
    for (int e = 0; e < o->ne; ++e) {
        double m = 0.0;
        for (int k = 0; k < 3; ++k) {
            int va = o->tri[3 * e + (k + 1) % 3], vb = o->tri[3 * e + (k + 2) % 3];
            double X = 0.5 * (o->vx[va] + o->vx[vb]), Y = 0.5 * (o->vy[va] + o->vy[vb]);
            int nb = o->nb[3 * e + k];
            double j = 0.0;
            if (nb >= 0) j = fabs(xi_p1_at(o, e, c, X, Y) - xi_p1_at(o, nb, c, X, Y));
            else if (o->btype[3 * e + k] == 1) j = fabs(xi_p1_at(o, e, c, X, Y) - xt);
            if (j > m) m = j;
        }
        I[e] = m;
    }
    return 0;
}

/* new order from the indicator: p_max if I >= tau, p_max-1 if I >= tau/10,
 * ..., never below p_lo; modes above the new K are dropped (L2 projection
 * for a hierarchical orthonormal basis) and new modes start at zero */
int orc_adapt(void *h, double t, double *c, double tau, int p_lo, int p_hi)
{
    orc *o = (orc *)h;
    double *I = malloc(sizeof(double) * o->ne);
    orc_indicator(h, t, c, I);
    for (int e = 0; e < o->ne; ++e) {
        int pn = p_lo;
        double thr = tau;
        for (int pp = p_hi; pp > p_lo; --pp) {
            if (I[e] >= thr) { pn = pp; break; }
            thr /= 10.0;
        }
        o->p[e] = pn;
        int Ke = K_OF_P[pn];
        for (int j = 0; j < 3; ++j)
            for (int i = Ke; i < o->K; ++i) c[(size_t)e * 3 * o->K + j * o->K + i] = 0.0;
    }
    free(I);
    return 0;
}

/* ------------------------------------------------------------------ */
/* SSP-RK2, Shu-Osher form:                                            */
/*   c1 = cn + dt L(cn, tn);  c_{n+1} = cn/2 + (c1 + dt L(c1, tn+dt))/2 */
/* ------------------------------------------------------------------ */
int orc_step(void *h, int nsteps, double dt, double t0, double *c, int adapt, double tau,
             int p_lo, int p_hi)
{
    orc *o = (orc *)h;
    size_t n = (size_t)o->ne * 3 * o->K;
    double *c1 = malloc(sizeof(double) * n), *L = malloc(sizeof(double) * n);
    int rc = 0;
    double t = t0;
    for (int s = 0; s < nsteps && rc == 0; ++s) {
        if (adapt) orc_adapt(h, t, c, tau, p_lo, p_hi);
        if ((rc = orc_rhs(h, t, c, L))) break;
        for (size_t i = 0; i < n; ++i) c1[i] = c[i] + dt * L[i];
        if (o->h_min > 0.0) orc_depth_limit(h, c1, o->h_min);
        if (!depth_ok(o, c1)) { rc = -4; break; }
        if ((rc = orc_rhs(h, t + dt, c1, L))) break;
        for (size_t i = 0; i < n; ++i) c[i] = 0.5 * c[i] + 0.5 * (c1[i] + dt * L[i]);
        if (o->h_min > 0.0) orc_depth_limit(h, c, o->h_min);
        if (!depth_ok(o, c)) { rc = -4; break; }
        t = t0 + (s + 1) * dt;
    }
    free(c1);
    free(L);
    return rc;
}

/* total water volume above the datum: sum_e int xi = sum_e xi_1 sqrt(area) */
double orc_mass(void *h, const double *c)
{
    orc *o = (orc *)h;
    double m = 0.0;
    for (int e = 0; e < o->ne; ++e) m += c[(size_t)e * 3 * o->K] * sqrt(0.5 * o->det[e]);
    return m;
}

/* ------------------------------------------------------------------ */
/* Input preparation: L2 projection of point values (n1 x n1 Duffy rule) */
/* ------------------------------------------------------------------ */
int orc_quad_points(void *h, int n1, double *xy)
{
    orc *o = (orc *)h;
    if (n1 < 1 || n1 > 16) return -1;
    tri_rule R;
    make_tri_rule(n1, &R);
    for (int e = 0; e < o->ne; ++e) {
        int a = o->tri[3 * e], b = o->tri[3 * e + 1], cc = o->tri[3 * e + 2];
        for (int q = 0; q < R.n; ++q) {
            double x = R.x[q], y = R.y[q];
            xy[((size_t)e * R.n + q) * 2 + 0] = o->vx[a] + x * (o->vx[b] - o->vx[a]) + y * (o->vx[cc] - o->vx[a]);
            xy[((size_t)e * R.n + q) * 2 + 1] = o->vy[a] + x * (o->vy[b] - o->vy[a]) + y * (o->vy[cc] - o->vy[a]);
        }
    }
    return 0;
}

/* vals[e][q][j]: field j at point q of element e; c_out[e][j][i] = int f_j phi_ei */
int orc_project(void *h, int n1, const double *vals, double *c)
{
    orc *o = (orc *)h;
    if (n1 < 1 || n1 > 16) return -1;
    tri_rule R;
    make_tri_rule(n1, &R);
    const int K = o->K;
    for (int e = 0; e < o->ne; ++e) {
        int Ke = K_OF_P[o->p[e]];
        double s = sqrt(o->det[e]);
        double *ce = c + (size_t)e * 3 * K;
        for (int i = 0; i < 3 * K; ++i) ce[i] = 0.0;
        for (int q = 0; q < R.n; ++q) {
            double phi[KMAX];
            basis_eval(Ke, R.x[q], R.y[q], phi, NULL, NULL);
            double w = R.w[q] * o->det[e];
            for (int j = 0; j < 3; ++j) {
                double f = vals[((size_t)e * R.n + q) * 3 + j];
                for (int i = 0; i < Ke; ++i) ce[j * K + i] += w * f * phi[i] / s;
            }
        }
    }
    return 0;
}

/* point evaluation of the discrete fields: out[j] = c_Delta_j(x,y), j<3; out[3..4] = u, v */
int orc_eval(void *h, const double *c, int e, double x, double y, double *out)
{
    orc *o = (orc *)h;
    double xh, yh, phi[KMAX];
    to_ref(o, e, x, y, &xh, &yh);
    eval_fields(o, e, c, o->u, xh, yh, phi, out, out + 3);
    return 0;
}

/* reference basis values (for the basis pins) */
int orc_basis(int K, double x, double y, double *phi, double *dx, double *dy)
{
    if (K < 1 || K > KMAX) return -1;
    build_basis();
    basis_eval(K, x, y, phi, dx, dy);
    return 0;
}

void orc_basis_coeffs(double *A)
{
    build_basis();
    memcpy(A, BASIS_A, sizeof(BASIS_A));
}

int orc_neighbours(void *h, int *nb, int *btype)
{
    orc *o = (orc *)h;
    memcpy(nb, o->nb, sizeof(int) * 3 * o->ne);
    memcpy(btype, o->btype, sizeof(int) * 3 * o->ne);
    return 0;
}
