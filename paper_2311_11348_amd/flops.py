"""Algorithmic floating-point work of one RK stage of one element.

The quadrature-free form contracts per-element coefficient vectors with the
reference tensors of ``csrc/gen_tables.py`` (Sec. "Quadrature-free DG
formulation of the shallow water equations", eq. (mass_basis) and the same
tensor algebra for the momentum rows; the edge term with the Lax-Friedrichs
flux of (eq:lambda); the truncated u H = q of Sec. "Algorithmic adaptation:
order separation").  This module counts the arithmetic of those contractions
with the tensors' exact zero patterns (an FMA is two operations, a multiply,
add or compare one), each interior edge flux once (one and a half edges per
element on a triangulation), for a uniform-order element: the figure a
compute roofline is priced with.  It counts operations; it evaluates none.
"""
from __future__ import annotations

import functools
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


@functools.lru_cache(maxsize=1)
def _tables():
    sys.path.insert(0, os.path.join(HERE, "csrc"))
    try:
        import gen_tables
        return gen_tables.build()
    finally:
        sys.path.pop(0)


def _nz(x) -> int:
    return int(x != 0.0)


@functools.lru_cache(maxsize=None)
def stage_flops(p: int, edges_per_element: float = 1.5) -> dict:
    """Operations of one stage of one element of order p, by part; ``fp64``
    is the part every precision does in FP64 (bathymetry terms)."""
    T = _tables()
    C, D, R, G = T["C"], T["D"], T["R"], T["G"]
    DEG = [0, 1, 1, 2, 2, 2, 3, 3, 3, 3]
    K = (p + 1) * (p + 2) // 2
    KM = p * (p + 1) // 2
    NT = p + 1
    out = {}
    # ---- volume: project the flux products onto P^{p-1} with C, apply D
    vol = vol64 = 0
    for m in range(KM):
        for i in range(K):
            row = sum(_nz(C[m][i][j]) for j in range(K))
            if row == 0:
                continue
            vol += 3 * 2 * row            # C-row contractions of u, v, xi
            vol += 5 * 2                  # U u, U v, V u, V v, xi xi accumulations
            vol64 += 2 * sum(_nz(C[m][i][j]) for j in range(3)) + 2   # xi h_b, FP64
        vol += 2 * 2 + 2                  # pressure into the two diagonal rows, F_W
    vol += 3 * KM * 2 * 3                 # B^-1 times the flux for each row and derivative
    for q in range(K):
        nzd = sum(_nz(D[0][q][m]) + _nz(D[1][q][m]) for m in range(KM))
        vol += 3 * 2 * nzd                # D contractions, three rows
        vol64 += 2 * 2 * nzd              # bathymetry part of the two momentum rows
    vol64 += 4 * KM
    out["volume"] = vol
    # ---- source: Coriolis, friction, g xi grad h_b
    out["source"] = 4 * 2 * K + 8
    src64 = 2 * 2 * K + 10
    # ---- edge fluxes (per edge): traces of both sides, normal parts,
    #      penalty, 1D products, flux assembly
    tr = 0
    for k in range(3):
        tr += sum(_nz(R[k][n][c]) for n in range(K) for c in range(NT) if c <= DEG[n])
    tr = 2 * 5 * 2 * tr / 3.0             # five fields, both sides, averaged over local edges
    prod = sum(_nz(G[c][a][b]) for c in range(NT) for a in range(NT) for b in range(NT))
    flux = tr + 2 * 2 * 3 * NT + 20       # normal parts of u and q on both sides, penalty
    flux += 6 * 2 * prod + NT * 14        # xi^2, U u_n, V u_n on both sides; LF assembly
    edge64 = 2 * sum(_nz(G[c][a][b]) for c in range(NT) for a in range(NT) for b in range(2)) + 3 * NT
    out["edge_flux"] = flux * edges_per_element
    # ---- lifting each of the element's three edge fluxes onto its test functions
    lift = 0
    for k in range(3):
        lift += sum(_nz(R[k][q][c]) for q in range(K) for c in range(NT))
    out["edge_lift"] = 3 * 2 * lift + 3 * 3 * NT
    lift64 = 2 * 2 * lift
    # ---- RK combine (second stage average) and u H = q by LDL^T
    out["rk"] = 3 * K * 3
    asm = 0
    for i in range(K):
        for j in range(i + 1):
            kt = (max(DEG[i], DEG[j]) + 1) * (max(DEG[i], DEG[j]) + 2) // 2
            asm += 2 * sum(_nz(C[n][i][j]) for n in range(kt)) + 2
    ldl = sum(2 * j + 1 + (K - j - 1) * (2 * j + 1) for j in range(K))
    solve = 2 * (K * (K - 1)) + 2 * K + 2 * (K * (K - 1))
    out["u_solve"] = asm + ldl + solve
    out["geometry"] = 40
    out["fp64"] = vol64 + src64 + edge64 * edges_per_element + lift64
    out["total"] = sum(v for k, v in out.items() if k not in ("fp64",))
    return out
