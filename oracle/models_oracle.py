"""FP64 oracle: matrix powers under the linear and skip-s iterative models.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Sec. 3.2 and Table 1 (matrix-powers column) define three iterative models
for P_k = A^k:

    linear       P_1 = A,  P_i = A P_{i-1}                 i = 2, 3, ..., k
    exponential  P_1 = A,  P_i = P_{i/2} P_{i/2}           i = 2, 4, ..., k
    skip-s       exponential up to P_s, then P_i = P_s P_{i-s}
                                                            i = 2s, 3s, ..., k

Each stored P_i is a product P_a P_b of two earlier stored matrices
(linear: a = 1, b = i - 1; skip: a = s, b = i - s for i > s; exponential:
a = b = i/2).  App. A gives the factored deltas of every model for
Delta A = U V^T with Delta P_i = U_i V_i^T, from the OLD matrices:

    U_i = [ U_a,  P_a U_b + U_a (V_a^T U_b) ]
    V_i = [ P_b^T V_a,  V_b ]

(the linear model with U_1, V_1 in place of U_a, V_a and A = P_1; the
skip model with U_s, V_s), widths i * r.  IncrLin and IncrSkip-s apply them
to every stored matrix after all factors are formed, as IncrExp does.
"""

from __future__ import annotations

import numpy as np

from .linview_oracle import OpCounter, levels


def model_steps(model: str, k: int, s: int | None = None) -> list[tuple[int, int, int]]:
    """The products (i, a, b), P_i = P_a P_b, of a model in evaluation order
    (Sec. 3.2, Table 1).  Linear: any k >= 1.  Exponential: k a power of
    two.  Skip-s: s a power of two dividing k (s = 1 is the linear model,
    s = k the exponential one)."""
    if model == "lin":
        if k < 1:
            raise ValueError("k must be >= 1")
        return [(i, 1, i - 1) for i in range(2, k + 1)]
    if model == "exp":
        return [(i, i // 2, i // 2) for i in levels(k)[1:]]
    if model == "skip":
        if s is None or s < 1 or (s & (s - 1)) != 0 or k % s != 0:
            raise ValueError(f"skip model needs s a power of two dividing k, got s={s}, k={k}")
        steps = [(i, i // 2, i // 2) for i in levels(s)[1:]]
        steps += [(i, s, i - s) for i in range(2 * s, k + 1, s)]
        return steps
    raise ValueError(f"unknown model {model!r}")


def stored_powers(model: str, k: int, s: int | None = None) -> list[int]:
    """The matrices a model materializes: 1 and every product's result."""
    return [1] + [i for i, _, _ in model_steps(model, k, s)]


def reeval_model(A: np.ndarray, model: str, k: int, s: int | None = None) -> dict[int, np.ndarray]:
    """Re-evaluation of every stored matrix by the model's products
    (Table 1): P_1 = A, then P_i = P_a P_b in order."""
    P = {1: np.asarray(A, dtype=np.float64).copy()}
    for i, a, b in model_steps(model, k, s):
        P[i] = P[a] @ P[b]
    return P


def incr_model_factors(P: dict[int, np.ndarray], U: np.ndarray, V: np.ndarray, model: str, k: int,
                       s: int | None = None, counter: OpCounter | None = None):
    """Factored deltas of every stored matrix (App. A, the model's rule in
    the module docstring), all from the old P.  Operation counts follow the
    convention of App. A (OpCounter).  Returns (dU, dV)."""
    c = counter if counter is not None else OpCounter()
    dU = {1: np.asarray(U, dtype=np.float64)}
    dV = {1: np.asarray(V, dtype=np.float64)}
    for i, a, b in model_steps(model, k, s):
        Ua, Va, Ub, Vb = dU[a], dV[a], dU[b], dV[b]
        G = c.mm(Va.T, Ub)                       # V_a^T U_b
        Z = c.add(c.mm(P[a], Ub), c.mm(Ua, G))   # P_a U_b + U_a (V_a^T U_b)
        Y = c.mm(P[b].T, Va)                     # P_b^T V_a
        dU[i] = np.hstack([Ua, Z])
        dV[i] = np.hstack([Y, Vb])
    return dU, dV


def incr_update_model(P: dict[int, np.ndarray], U: np.ndarray, V: np.ndarray, model: str, k: int,
                      s: int | None = None, counter: OpCounter | None = None) -> dict[int, np.ndarray]:
    """IncrLin / IncrSkip-s (or IncrExp) step: all factors from the old
    matrices, then P_i += U_i V_i^T for every stored i.  Returns the new
    dict; the input is not modified."""
    c = counter if counter is not None else OpCounter()
    dU, dV = incr_model_factors(P, U, V, model, k, s, c)
    return {i: c.rank_update(P[i], dU[i], dV[i]) for i in P}


def paper_cost(model: str, n: int, k: int, s: int | None = None) -> int:
    """Operation count of one rank-1 refresh of all stored matrices as
    App. A states it in closed form (linear and exponential models; for the
    skip model the exact sum whose order App. A gives, exponential part up to
    s plus the skip products)."""
    if model == "lin":
        return n * n * (k * k + k - 1) + 3 * n * k * (k - 1) // 2
    if model == "exp":
        return n * n * (4 * k - 3) + n * (k - 1) * (2 * k + 5) // 3
    if model == "skip":
        K = k // s
        exp_part = n * n * (4 * s - 3) + n * (s - 1) * (2 * s + 5) // 3
        return exp_part + n * n * (k * k // s + k - 2 * s) + (2 * s + 1) * n * s * K * (K - 1) // 2
    raise ValueError(model)
