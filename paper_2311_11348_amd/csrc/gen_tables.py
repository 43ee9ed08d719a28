"""Generate ``swe_tables.h``: exact reference-element tensors of the method.

The quadrature-free scheme integrates products of basis functions exactly with
precomputed integrals (Sec. "Algorithmic adaptation: order separation",
eq. (mass_basis), and the code-generation section, which builds them
symbolically).  Here they are built in exact rational arithmetic:

* basis: Gram-Schmidt of 1, x, y, x^2, xy, y^2, x^3, x^2y, xy^2, y^3 on the
  reference triangle T = {x, y >= 0, x + y <= 1}, kept as rational orthogonal
  polynomials psi_i with rational norms N_i, phi_i = psi_i / sqrt(N_i), so it
  is hierarchical and orthonormal (K(p) = 1, 3, 6, 10);
* C[m][i][j] = int_T phi_m phi_i phi_j          (products, u H = q)
* D[k][q][m] = int_T d_k phi_q phi_m             (volume derivative matrix)
* R[k][q][a] = int_0^1 phi_q(edge_k(t)) L_a(t)   (traces on local edge k)
* G[c][a][b] = int_0^1 L_a L_b L_c               (1D products on an edge)
* W[n][v]    = int_T lambda_v phi_n              (P1 bathymetry -> modes)
* PMID[k][n] = phi_n(midpoint of edge k)         (P1 part at edge midpoints)
* PCHK[j][n] = phi_n at the three vertices, then the three edge midpoints
                                                (points of the minimum-depth control)
* a 36-point collapsed Gauss rule with phi values, for projecting initial data.
Local edge k joins reference vertices k+1 and k+2 (vertices (0,0), (1,0),
(0,1)), parametrised by t from vertex k+1 to vertex k+2; L_a are the
orthonormal Legendre polynomials on [0, 1].

Every constant is exact (rational times the square root of a rational) before
it is rounded once to the nearest double.
"""
from __future__ import annotations

import math
import os
import sys
from decimal import Decimal, getcontext
from fractions import Fraction as F

getcontext().prec = 60

MONO = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3)]
KMAX = 10
DEG = [a + b for a, b in MONO]
VERT = [(F(0), F(0)), (F(1), F(0)), (F(0), F(1))]


# polynomials in (x, y): dict {(a, b): Fraction}
def padd(p, q, s=F(1)):
    r = dict(p)
    for k, v in q.items():
        r[k] = r.get(k, F(0)) + s * v
    return {k: v for k, v in r.items() if v != 0}


def pmul(p, q):
    r = {}
    for (a, b), v in p.items():
        for (c, d), w in q.items():
            k = (a + c, b + d)
            r[k] = r.get(k, F(0)) + v * w
    return {k: v for k, v in r.items() if v != 0}


def pscale(p, s):
    return {k: v * s for k, v in p.items()}


def pdiff(p, var):
    r = {}
    for (a, b), v in p.items():
        if var == 0 and a > 0:
            r[(a - 1, b)] = r.get((a - 1, b), F(0)) + a * v
        if var == 1 and b > 0:
            r[(a, b - 1)] = r.get((a, b - 1), F(0)) + b * v
    return r


def tri_int(p):
    """int_T x^a y^b = a! b! / (a + b + 2)!"""
    return sum((v * F(math.factorial(a) * math.factorial(b), math.factorial(a + b + 2))
                for (a, b), v in p.items()), F(0))


# univariate polynomials in t: list of Fractions (coefficient of t^i)
def uadd(p, q, s=F(1)):
    n = max(len(p), len(q))
    return [(p[i] if i < len(p) else F(0)) + s * (q[i] if i < len(q) else F(0)) for i in range(n)]


def umul(p, q):
    r = [F(0)] * (len(p) + len(q) - 1)
    for i, a in enumerate(p):
        for j, b in enumerate(q):
            r[i + j] += a * b
    return r


def uint01(p):
    return sum((v / (i + 1) for i, v in enumerate(p)), F(0))


def restrict(p, k):
    """psi(edge_k(t)) as a polynomial in t."""
    a0, b0 = VERT[(k + 1) % 3]
    a1, b1 = VERT[(k + 2) % 3]
    X = [a0, a1 - a0]
    Y = [b0, b1 - b0]
    out = [F(0)]
    for (a, b), v in p.items():
        term = [v]
        for _ in range(a):
            term = umul(term, X)
        for _ in range(b):
            term = umul(term, Y)
        out = uadd(out, term)
    return out


def shifted_legendre(n):
    """P_n(2t - 1) with rational coefficients (unnormalised, P_n(1) = 1)."""
    P = [[F(1)], [F(-1), F(2)]]
    for k in range(1, n):
        # (k+1) P_{k+1} = (2k+1)(2t-1) P_k - k P_{k-1}
        a = umul([F(-1), F(2)], P[k])
        nxt = uadd(pscale_u(a, F(2 * k + 1, k + 1)), pscale_u(P[k - 1], F(-k, k + 1)))
        P.append(nxt)
    return P[: n + 1]


def pscale_u(p, s):
    return [v * s for v in p]


class Exact:
    """r * sqrt(s) with rationals r, s >= 0."""

    def __init__(self, r, s=F(1)):
        self.r, self.s = F(r), F(s)

    def to_double(self):
        if self.r == 0:
            return 0.0
        d = Decimal(self.r.numerator) / Decimal(self.r.denominator)
        d *= (Decimal(self.s.numerator) / Decimal(self.s.denominator)).sqrt()
        return float(d)


def build():
    psi, N = [], []
    for i in range(KMAX):
        m = {MONO[i]: F(1)}
        v = dict(m)
        for j in range(i):
            ip = tri_int(pmul(m, psi[j]))
            v = padd(v, psi[j], -ip / N[j])
        psi.append(v)
        N.append(tri_int(pmul(v, v)))
    T = {}
    # C[m][i][j]
    C = [[[Exact(tri_int(pmul(pmul(psi[m], psi[i]), psi[j])), 1 / (N[m] * N[i] * N[j])).to_double()
           for j in range(KMAX)] for i in range(KMAX)] for m in range(KMAX)]
    D = [[[Exact(tri_int(pmul(pdiff(psi[q], k), psi[m])), 1 / (N[q] * N[m])).to_double()
           for m in range(KMAX)] for q in range(KMAX)] for k in range(2)]
    PL = shifted_legendre(3)
    R = [[[Exact(uint01(umul(restrict(psi[q], k), PL[a])), F(2 * a + 1) / N[q]).to_double()
           for a in range(4)] for q in range(KMAX)] for k in range(3)]
    G = [[[Exact(uint01(umul(umul(PL[a], PL[b]), PL[c])), F((2 * a + 1) * (2 * b + 1) * (2 * c + 1))).to_double()
           for b in range(4)] for a in range(4)] for c in range(4)]
    lam = [{(0, 0): F(1), (1, 0): F(-1), (0, 1): F(-1)}, {(1, 0): F(1)}, {(0, 1): F(1)}]
    W = [[Exact(tri_int(pmul(lam[v], psi[n])), 1 / N[n]).to_double() for v in range(3)] for n in range(3)]
    PMID = []
    for k in range(3):
        t = restrict_point(k, F(1, 2))
        PMID.append([Exact(peval(psi[n], t), 1 / N[n]).to_double() for n in range(3)])
    pts = [VERT[v] for v in range(3)] + [restrict_point(k, F(1, 2)) for k in range(3)]
    PCHK = [[Exact(peval(psi[n], pt), 1 / N[n]).to_double() for n in range(KMAX)] for pt in pts]
    T.update(C=C, D=D, R=R, G=G, W=W, PMID=PMID, PCHK=PCHK)
    # projection rule: collapsed Gauss-Legendre 6x6 (degree 10), double precision is enough
    import numpy as np
    tg, wg = np.polynomial.legendre.leggauss(6)
    tg, wg = 0.5 * (tg + 1.0), 0.5 * wg
    qx, qy, qw = [], [], []
    for i in range(6):
        for j in range(6):
            qx.append(tg[i])
            qy.append(tg[j] * (1 - tg[i]))
            qw.append(wg[i] * wg[j] * (1 - tg[i]))
    qphi = [[sum(float(v) * qx[p] ** a * qy[p] ** b for (a, b), v in psi[n].items()) / math.sqrt(float(N[n]))
             for n in range(KMAX)] for p in range(36)]
    T.update(QX=qx, QY=qy, QW=qw, QPHI=qphi)
    return T


def restrict_point(k, t):
    a0, b0 = VERT[(k + 1) % 3]
    a1, b1 = VERT[(k + 2) % 3]
    return (a0 + t * (a1 - a0), b0 + t * (b1 - b0))


def peval(p, pt):
    x, y = pt
    return sum((v * x ** a * y ** b for (a, b), v in p.items()), F(0))


def fmt(v):
    if v == 0.0:
        return "0.0"
    return repr(float(v))


def nested(a):
    if isinstance(a, list):
        return "{" + ", ".join(nested(x) for x in a) + "}"
    return fmt(a)


def emit(T, path):
    lines = [
        "// Generated by gen_tables.py from exact rational arithmetic. Do not edit.",
        "// Reference triangle {x,y >= 0, x+y <= 1}; hierarchical orthonormal basis",
        "// (Gram-Schmidt of 1,x,y,x^2,xy,y^2,x^3,x^2y,xy^2,y^3); local edge k joins",
        "// reference vertices k+1 and k+2, parameter t in [0,1] from k+1 to k+2;",
        "// L_a = orthonormal Legendre polynomials on [0,1].",
        "#pragma once",
        "",
        "#define SWET_K_OF_P {1, 3, 6, 10}",
        "#define SWET_DEG {" + ", ".join(str(d) for d in DEG) + "}",
        "// C[m][i][j] = int phi_m phi_i phi_j",
        "#define SWET_C " + nested(T["C"]),
        "// D[k][q][m] = int d(phi_q)/d(x_k) phi_m",
        "#define SWET_D " + nested(T["D"]),
        "// R[k][q][a] = int_0^1 phi_q(edge_k(t)) L_a(t) dt",
        "#define SWET_R " + nested(T["R"]),
        "// G[c][a][b] = int_0^1 L_a L_b L_c dt",
        "#define SWET_G " + nested(T["G"]),
        "// W[n][v] = int lambda_v phi_n (barycentric lambda_v of vertex v)",
        "#define SWET_W " + nested(T["W"]),
        "// PMID[k][n] = phi_n at the midpoint of edge k",
        "#define SWET_PMID " + nested(T["PMID"]),
        "// PCHK[j][n] = phi_n at reference vertex j (j < 3), at the midpoint of edge j - 3 (j >= 3)",
        "#define SWET_PCHK " + nested(T["PCHK"]),
        "// 36-point collapsed Gauss rule (degree 10) for projecting point data",
        "#define SWET_NQP 36",
        "#define SWET_QX " + nested(T["QX"]),
        "#define SWET_QY " + nested(T["QY"]),
        "#define SWET_QW " + nested(T["QW"]),
        "#define SWET_QPHI " + nested(T["QPHI"]),
        "",
    ]
    text = "\n".join(lines)
    with open(path, "w") as f:
        f.write(text)
    return text


if __name__ == "__main__":
    out = sys.argv[1] if len(sys.argv) > 1 else os.path.join(os.path.dirname(os.path.abspath(__file__)), "swe_tables.h")
    emit(build(), out)
    print("wrote", out)
