"""Cost models of the Uzawa multigrid (test infrastructure, like the rest of
the oracle): operator evaluations weighted by level size, the textbook
multigrid efficiency of FMG, and the memory of the method.

Each function writes out the closed form the paper gives, in its notation.
"""
from __future__ import annotations


def level_weight(l: int, L: int) -> float:
    """Work of level l relative to the finest level L under standard 3D
    coarsening: 8^(l-L) (Section 4.1, memory model; Section 4.2)."""
    return 8.0 ** (l - L)


def uzawa_ops_per_level(L: int, l: int, nu: int = 3, variable: bool = True) -> dict:
    """Operator evaluations of one V-cycle on level l (Section 4.2): each
    Uzawa step applies A twice (forward and backward Gauss-Seidel), B twice
    and C once (eq. Uzawa_smooth); a V(nu, nu) cycle makes 2 nu steps, the
    variable cycle 2 (nu + 2 (L - l)); the residual adds one A and, through
    B and B^T, the B count (hence the '+1' and '+2' of the paper's sums)."""
    steps = 2 * (nu + (2 * (L - l) if variable else 0))
    return {"A": 2 * steps + 1, "B": 2 * steps + 2, "C": steps + 1}


def n_op(block: str, L: int, n_I: int, nu: int = 3) -> float:
    """Weighted operator evaluations per block (eq. op_count) for n_I
    variable V(nu, nu) cycles: n_I sum_l 8^(l-L) n_op,l.  The paper's sums
    for A and B use 4 (3 + 2 (L - l)) + 1 and + 2; for C it states half of
    B."""
    tot = 0.0
    for l in range(L + 1):
        per = 4 * (nu + 2 * (L - l))
        if block == "A":
            cnt = per + 1
        elif block == "B":
            cnt = per + 2
        elif block == "C":
            cnt = (per + 2) / 2.0
        else:
            raise ValueError(block)
        tot += level_weight(l, L) * cnt
    return n_I * tot


def wu_per_smoothing_step() -> float:
    """One Uzawa smoothing step with its residual part applies A_1 twice
    (6 blocks), B twice (6 blocks) and C once (1 block) of the 10 blocks of
    one K application: 13/10 WU (Section 5)."""
    return (2 * 3 + 2 * 3 + 1) / 10.0


def e_tme(nu: int = 2, L_max: int = 60) -> float:
    """E_TME of FMG with one variable V(nu, nu) cycle per level (Section 5):
    the double sum over the FMG levels k and the V-cycle levels l of
    8^-k 8^(l-L) (2 (nu + 2 (L - l)) 13/10 + 1), the '+1' being the residual
    per level, in the limit of many levels (L_max terms; the terms decay like
    8^-k)."""
    wu = wu_per_smoothing_step()
    L = L_max
    inner = sum(8.0 ** (l - L) * (2 * (nu + 2 * (L - l)) * wu + 1.0) for l in range(1, L + 1))
    return sum(8.0 ** (-k) for k in range(L)) * inner


def memory_bytes(L: int, vectors: int = 3, bytes_per_value: int = 8) -> float:
    """m_t of eq. (memory): 3 vectors (unknowns, right-hand side, residual)
    of n_{L,u} + n_{L,p} doubles on every level, the levels weighted by
    sum_l 8^(l-L).  The count n_{L,u} + n_{L,p} = 4 (n - 1)^3 on the unit
    cube with n = 2^(L+2) intervals per edge (the paper's level L is R = L+2
    refinements of the 6 macro tetrahedra; its DoF column counts the interior
    lattice points)."""
    n = 2 ** (L + 2)
    dofs = 4 * (n - 1) ** 3
    return vectors * dofs * sum(level_weight(l, L) for l in range(L + 1)) * bytes_per_value


def velocity_cycle_ops(L: int, nu1: int, nu2: int) -> float:
    """Weighted A evaluations of one velocity V(nu1, nu2) cycle with (FHGS,
    BHGS) smoothing (Section 3.5, Table "settings"): a forward or backward
    sweep over all colours applies A once, the residual before restriction
    once more, on every level (the same per-level convention as the UMG sums
    of Section 4.2, which include level 0)."""
    return sum(level_weight(l, L) * (nu1 + nu2 + 1) for l in range(L + 1))


def pminres_ops(L: int, iterations: int, nu: int = 1) -> dict:
    """Operator evaluations of block-diagonal PMINRES (Section 3.2): the
    initial residual and every iteration apply K once (A once, B and B^T,
    C once) and the preconditioner once (a velocity V(nu, nu) cycle and the
    lumped mass M)."""
    k = iterations + 1
    return {"A": k * (1.0 + velocity_cycle_ops(L, nu, nu)), "B": 2.0 * k, "C": float(k),
            "M": float(k)}
