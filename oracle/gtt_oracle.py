"""Plain FP64 CPU oracle for the generalized tensor transform (GTT).

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the CPU
baseline leg of the benchmark may import this module.  The product path (the
HIP library and its Python binding) never imports, calls or links anything
here, and nothing here imports the product path.

Every routine is written for a reader holding the paper
(Shukla & Vedula, "Generalized tensor transforms and their applications in
classical and quantum computing"), not for speed.  Floating point is float64 /
complex128; integer transforms use exact Python/NumPy int64 arithmetic and
wrap to two's-complement int32 only at the end.

Conventions used throughout (all from the paper):
  * an index k < b**n has base-b digits k = sum_j k_j b**j, digit 0 being the
    least significant (§2.1, notation);
  * W[i, j] is row i, column j, 0-based (§2.1);
  * the GTT matrix is G_N = W kron W kron ... kron W (n factors) (§2.6,
    Def. 2.4), whose entries are G_N(p, q) = prod_j W[p_j, q_j] (§2.6, the
    product formula after Def. 2.4).

Pins: every function here is pinned in the CPU tests against something other
than itself (paper-printed values, textbook matrices, library FFTs, brute
force, finite differences).  No function in this file is "parity unpinned".
"""
from __future__ import annotations

import math
from typing import Sequence

import numpy as np

__all__ = [
    "digits",
    "basis_function",
    "gtt_matrix_from_basis",
    "kron_power",
    "kron_list",
    "dense",
    "entry",
    "row",
    "rows",
    "fastgtt_rec",
    "staged",
    "staged_mixed",
    "adjoint",
    "grad",
    "fd_grad",
    "grad_mixed",
    "fd_grad_mixed",
    "staged_int32",
    "adjoint_int32",
    "sylvester_hadamard",
    "natural_filter",
    "topk_compress",
    "kept_energy",
    "fidelity",
]


# ---------------------------------------------------------------------------
# Digits (§2.1)
# ---------------------------------------------------------------------------
def digits(k: int, b: int, n: int) -> list[int]:
    """Base-b digits [k_0, k_1, ..., k_{n-1}] of k, least significant first (§2.1)."""
    out = []
    for _ in range(n):
        out.append(k % b)
        k //= b
    return out


# ---------------------------------------------------------------------------
# Construction 1: sampled basis functions (§2.2 recursion, §2.6 discretization)
# ---------------------------------------------------------------------------
def basis_function(j: int, x: float, W: np.ndarray, n: int) -> complex:
    """f_j^{(b^n)}(x) from the recursive definition of §2.2.

    Base case n = 0: f_0^{(1)}(x) = 1 on [0, 1).  For n >= 1 the value is
    W[floor(b x), floor(j / b^{n-1})] times f_{j mod b^{n-1}}^{(b^{n-1})}({b x}),
    where {.} is the fractional part (§2.1).  Pure-Python recursion: only for
    small n.
    """
    b = W.shape[0]
    if not (0.0 <= x < 1.0):
        return 0.0
    if n == 0:
        return 1.0
    bx = b * x
    row_i = int(math.floor(bx))
    top = b ** (n - 1)
    col_j = j // top
    return W[row_i, col_j] * basis_function(j % top, bx - math.floor(bx), W, n - 1)


def gtt_matrix_from_basis(W: np.ndarray, n: int) -> np.ndarray:
    """G_N(p, q) = f_q^{(N)}(x_p) at midpoints x_p = (2p+1)/(2N) (§2.6, discretization).

    This is an independent construction of the GTT matrix; the paper states it
    equals the Kronecker power of Def. 2.4.  Tiny N only.
    """
    b = W.shape[0]
    N = b ** n
    G = np.zeros((N, N), dtype=np.complex128)
    for p in range(N):
        xp = (2 * p + 1) / (2 * N)
        for q in range(N):
            G[p, q] = basis_function(q, xp, W, n)
    return G


# ---------------------------------------------------------------------------
# Construction 2: the definition G_N = W^{kron n} (§2.6, Def. 2.4)
# ---------------------------------------------------------------------------
def kron_power(W: np.ndarray, n: int) -> np.ndarray:
    """W kron W kron ... kron W with n factors (§2.6, Def. 2.4); n = 0 gives [[1]]."""
    G = np.ones((1, 1), dtype=np.result_type(W, np.float64))
    for _ in range(n):
        G = np.kron(G, W)
    return G


def kron_list(Ws: Sequence[np.ndarray]) -> np.ndarray:
    """Heterogeneous GTT matrix W_0 kron W_1 kron ... kron W_{n-1} (§2.6, remark on
    distinct factors).  The leftmost factor acts on the most significant digit."""
    G = np.ones((1, 1), dtype=np.complex128)
    for Wk in Ws:
        G = np.kron(G, Wk)
    return G


def dense(W: np.ndarray, x: np.ndarray, n: int) -> np.ndarray:
    """y = G_N x with the dense Kronecker matrix (Def. 2.4).  x: (N,) or (batch, N).
    Only for N <= 4096 (the dense matrix is N x N)."""
    G = kron_power(W, n)
    return np.asarray(x) @ G.T


# ---------------------------------------------------------------------------
# Construction 3: the entrywise product formula (§2.6, after Def. 2.4)
# ---------------------------------------------------------------------------
def entry(W: np.ndarray, p: int, q: int, n: int):
    """G_N(p, q) = prod_{j<n} W[p_j, q_j] with base-b digits of p and q."""
    b = W.shape[0]
    pd, qd = digits(p, b, n), digits(q, b, n)
    val = 1
    for j in range(n):
        val = val * W[pd[j], qd[j]]
    return val


def row(W: np.ndarray, p: int, n: int) -> np.ndarray:
    """Row p of G_N, built from the product formula: entry q is prod_j W[p_j, q_j].

    Written as a Kronecker product of the n row vectors W[p_j, :] (most
    significant digit leftmost), i.e. O(N) work per row.  Works at any N.
    """
    b = W.shape[0]
    pd = digits(p, b, n)
    r = np.ones(1, dtype=np.result_type(W, np.float64))
    for j in reversed(range(n)):            # digit n-1 is the leftmost factor
        r = np.kron(r, W[pd[j], :])
    return r


def rows(W: np.ndarray, x: np.ndarray, n: int, ps: Sequence[int]) -> np.ndarray:
    """y_p = sum_q G_N(p, q) x_q for the sampled indices ps (any N)."""
    x = np.asarray(x)
    return np.array([row(W, int(p), n) @ x for p in ps])


# ---------------------------------------------------------------------------
# Construction 4: Algorithm 1 (§3.1), recursive
# ---------------------------------------------------------------------------
def fastgtt_rec(x: np.ndarray, W: np.ndarray, n: int) -> np.ndarray:
    """FastGTT(x, W, n) as described in §3 / Alg. 1.

    Base case n = 1 returns W x.  Otherwise the vector is viewed as an
    (N/b) x b matrix X with X[p, q] = x[p b + q], Y = X W^T (W along the last
    digit), each of the b columns of Y is transformed recursively with n - 1
    digits, and the rows of the result are concatenated.  n = 0 is the
    identity (the base case of §2.2, N = 1).
    """
    x = np.asarray(x)
    b = W.shape[0]
    if n == 0:
        return x.copy()
    if n == 1:
        return W @ x
    N = b ** n
    X = x.reshape(N // b, b)
    Y = X @ W.T
    Z = np.zeros_like(Y, dtype=np.result_type(Y, W))
    for j in range(b):
        Z[:, j] = fastgtt_rec(Y[:, j], W, n - 1)
    return Z.reshape(N)


# ---------------------------------------------------------------------------
# Construction 5: staged mode-s passes (the straightforward staged algorithm)
# ---------------------------------------------------------------------------
def staged(W: np.ndarray, x: np.ndarray, n: int) -> np.ndarray:
    """y = G_N x as n passes; pass s applies W along base-b digit s (§3: each
    level of Alg. 1 is Y = X W^T along one digit; the levels commute because
    they act on different tensor factors of Def. 2.4).

    x: (N,) or (batch, N), any float/complex dtype; computed in float64 /
    complex128.  Order of passes: digit 0 first, as in Alg. 1.
    """
    W = np.asarray(W)
    b = W.shape[0]
    x = np.asarray(x)
    one = x.ndim == 1
    X = x.reshape(1, -1) if one else x
    batch, N = X.shape
    assert N == b ** n, "N must equal b**n"
    ct = np.complex128 if (np.iscomplexobj(W) or np.iscomplexobj(X)) else np.float64
    a = X.astype(ct)
    Wc = W.astype(ct)
    for s in range(n):
        # view as (batch, high digits, digit s, low digits)
        a = a.reshape(batch, b ** (n - 1 - s), b, b ** s)
        a = np.einsum("ij,zajk->zaik", Wc, a)
    a = a.reshape(batch, N)
    return a[0] if one else a


def staged_mixed(Ws: Sequence[np.ndarray], x: np.ndarray) -> np.ndarray:
    """Heterogeneous GTT W_0 kron ... kron W_{n-1} applied to x (§2.6, remark on
    distinct factors): factor k has size b_k and acts on the digit of the mixed
    radix index whose place value is prod_{m>k} b_m (the leftmost factor acts on
    the most significant digit), as in np.kron."""
    x = np.asarray(x)
    one = x.ndim == 1
    X = x.reshape(1, -1) if one else x
    batch, N = X.shape
    bs = [np.asarray(Wk).shape[0] for Wk in Ws]
    assert N == int(np.prod(bs))
    a = X.astype(np.complex128)
    for k, Wk in enumerate(Ws):
        hi = int(np.prod(bs[:k])) if k else 1
        lo = int(np.prod(bs[k + 1:])) if k + 1 < len(bs) else 1
        a = a.reshape(batch, hi, bs[k], lo)
        a = np.einsum("ij,zajk->zaik", np.asarray(Wk, dtype=np.complex128), a)
    a = a.reshape(batch, N)
    return a[0] if one else a


def adjoint(W: np.ndarray, y: np.ndarray, n: int) -> np.ndarray:
    """x = G_N^dagger y = (W^H)^{kron n} y, the inverse transform used by every
    application in §4 (G^dagger in the compression and filtering protocols)."""
    return staged(np.conj(np.asarray(W)).T, y, n)


# ---------------------------------------------------------------------------
# Gradients (the paper has no derivatives; convention stated here)
# ---------------------------------------------------------------------------
def grad(W: np.ndarray, x: np.ndarray, g: np.ndarray, n: int):
    """Gradients of L = Re <g, y> = Re sum_i conj(g_i) y_i with y = G_N x.

    <.,.> is the bra-ket inner product of §2.4 (conjugate-linear in its first
    argument).  Gradients follow PyTorch's convention dL/dRe(z) + i dL/dIm(z).

      gx = G_N^H g;
      gW = sum over stages s of sum over the fibres of digit s of c_s a_s^H,
    where a_s is the input of stage s (digits 0..s-1 already transformed) and
    c_s is the cotangent at its output (W^H applied along digits s+1..n-1 of g).

    Each stage's contribution is written out plainly: for every fibre
    (fixed values of all digits but s) the outer product c a^H is added.
    Works for any W (unitarity is not assumed).  x, g: (N,) or (batch, N).
    Returns (gx, gW).
    """
    W = np.asarray(W)
    b = W.shape[0]
    x = np.asarray(x)
    g = np.asarray(g)
    one = x.ndim == 1
    X = x.reshape(1, -1) if one else x
    Gc = g.reshape(1, -1) if one else g
    batch, N = X.shape
    ct = np.complex128 if (np.iscomplexobj(W) or np.iscomplexobj(X) or np.iscomplexobj(Gc)) else np.float64
    Wc = W.astype(ct)
    WH = np.conj(Wc).T
    # stage inputs a_0..a_{n-1}
    acts = []
    a = X.astype(ct)
    for s in range(n):
        acts.append(a.copy())
        a4 = a.reshape(batch, b ** (n - 1 - s), b, b ** s)
        a = np.einsum("ij,zajk->zaik", Wc, a4).reshape(batch, N)
    gW = np.zeros((b, b), dtype=ct)
    c = Gc.astype(ct)                    # cotangent at the output of stage n-1
    for s in reversed(range(n)):
        c4 = c.reshape(batch, b ** (n - 1 - s), b, b ** s)
        a4 = acts[s].reshape(batch, b ** (n - 1 - s), b, b ** s)
        # sum over batch z, high digits a, low digits k of c[., i, .] conj(a[., j, .])
        gW += np.einsum("zaik,zajk->ij", c4, np.conj(a4))
        c = np.einsum("ij,zajk->zaik", WH, c4).reshape(batch, N)
    gx = c
    return (gx[0] if one else gx), gW


def fd_grad(W: np.ndarray, x: np.ndarray, g: np.ndarray, n: int, h: float = 1e-6):
    """Central finite differences of L = Re <g, G_N x> with respect to every real
    and imaginary component of x and W; returns (gx, gW) in the convention
    dL/dRe + i dL/dIm.  The forward map is the dense Kronecker product, so
    this check shares nothing with `grad`.  Tiny N only."""
    W = np.asarray(W, dtype=np.complex128)
    x = np.asarray(x, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)

    def loss(Wv, xv):
        y = kron_power(Wv, n) @ xv
        return float(np.real(np.vdot(g, y)))

    gx = np.zeros_like(x)
    for i in range(x.size):
        for unit in (1.0, 1j):
            xp = x.copy(); xp[i] += h * unit
            xm = x.copy(); xm[i] -= h * unit
            d = (loss(W, xp) - loss(W, xm)) / (2 * h)
            gx[i] += d * unit
    gW = np.zeros_like(W)
    for i in range(W.shape[0]):
        for j in range(W.shape[1]):
            for unit in (1.0, 1j):
                Wp = W.copy(); Wp[i, j] += h * unit
                Wm = W.copy(); Wm[i, j] -= h * unit
                d = (loss(Wp, x) - loss(Wm, x)) / (2 * h)
                gW[i, j] += d * unit
    return gx, gW


def grad_mixed(Ws: Sequence[np.ndarray], x: np.ndarray, g: np.ndarray):
    """Gradients of L = Re <g, y> for the heterogeneous transform
    y = (W_0 kron ... kron W_{m-1}) x (§2.6, remark on distinct factors), in the
    convention of `grad`: gx = G^H g and, for every factor k separately,
    gW_k = sum over the fibres of factor k's digit of c_k a_k^H, where a_k is
    the input of the stage of factor k and c_k the cotangent at its output.
    The stages run in factor order 0..m-1, as in `staged_mixed` (factor k
    acts on the digit whose place value is prod_{m>k} b_m).
    Returns (gx, [gW_0, ..., gW_{m-1}])."""
    x = np.asarray(x)
    g = np.asarray(g)
    one = x.ndim == 1
    X = x.reshape(1, -1) if one else x
    Gc = g.reshape(1, -1) if one else g
    batch, N = X.shape
    bs = [np.asarray(Wk).shape[0] for Wk in Ws]
    assert N == int(np.prod(bs))
    Wc = [np.asarray(Wk, dtype=np.complex128) for Wk in Ws]

    def view(a, k):
        hi = int(np.prod(bs[:k])) if k else 1
        lo = int(np.prod(bs[k + 1:])) if k + 1 < len(bs) else 1
        return a.reshape(batch, hi, bs[k], lo)

    acts = []
    a = X.astype(np.complex128)
    for k in range(len(Ws)):
        acts.append(a.copy())
        a = np.einsum("ij,zajk->zaik", Wc[k], view(a, k)).reshape(batch, N)
    gWs = [None] * len(Ws)
    c = Gc.astype(np.complex128)
    for k in reversed(range(len(Ws))):
        c4 = view(c, k)
        gWs[k] = np.einsum("zaik,zajk->ij", c4, np.conj(view(acts[k], k)))
        c = np.einsum("ij,zajk->zaik", np.conj(Wc[k]).T, c4).reshape(batch, N)
    return (c[0] if one else c), gWs


def fd_grad_mixed(Ws: Sequence[np.ndarray], x: np.ndarray, g: np.ndarray, h: float = 1e-6):
    """Central finite differences of L = Re <g, (W_0 kron ... kron W_{m-1}) x>
    with respect to every real and imaginary component of x and of each W_k,
    through the dense Kronecker product (shares nothing with `grad_mixed`).
    Tiny N only.  Returns (gx, [gW_k])."""
    Ws = [np.asarray(Wk, dtype=np.complex128) for Wk in Ws]
    x = np.asarray(x, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128)

    def loss(ws, xv):
        return float(np.real(np.vdot(g, kron_list(ws) @ xv)))

    gx = np.zeros_like(x)
    for i in range(x.size):
        for unit in (1.0, 1j):
            xp = x.copy(); xp[i] += h * unit
            xm = x.copy(); xm[i] -= h * unit
            gx[i] += (loss(Ws, xp) - loss(Ws, xm)) / (2 * h) * unit
    gWs = []
    for k, Wk in enumerate(Ws):
        gk = np.zeros_like(Wk)
        for i in range(Wk.shape[0]):
            for j in range(Wk.shape[1]):
                for unit in (1.0, 1j):
                    wp = [w.copy() for w in Ws]; wp[k][i, j] += h * unit
                    wm = [w.copy() for w in Ws]; wm[k][i, j] -= h * unit
                    gk[i, j] += (loss(wp, x) - loss(wm, x)) / (2 * h) * unit
        gWs.append(gk)
    return gx, gWs


# ---------------------------------------------------------------------------
# Integer transform (exact, two's-complement wrap-around at the end)
# ---------------------------------------------------------------------------
def _wrap32(a: np.ndarray) -> np.ndarray:
    a = np.asarray(a, dtype=np.int64) & 0xFFFFFFFF
    return np.where(a >= 2 ** 31, a - 2 ** 32, a).astype(np.int32)


def staged_int32(W: np.ndarray, x: np.ndarray, n: int) -> np.ndarray:
    """Integer G_N x for an integer W (e.g. the unnormalized +-1 Hadamard of
    §2.6's Hadamard reduction), computed exactly as mode-s passes in int64 with
    reduction mod 2^32 after every stage (a ring homomorphism, so the result is
    the exact value mod 2^32), returned as two's-complement int32."""
    W = np.asarray(W, dtype=np.int64)
    b = W.shape[0]
    x = np.asarray(x)
    one = x.ndim == 1
    X = (x.reshape(1, -1) if one else x).astype(np.int64)
    batch, N = X.shape
    assert N == b ** n
    a = X
    for s in range(n):
        a = a.reshape(batch, b ** (n - 1 - s), b, b ** s)
        a = np.einsum("ij,zajk->zaik", W, a)
        a = a & 0xFFFFFFFF  # keep exact value mod 2^32 (no int64 overflow)
    out = _wrap32(a.reshape(batch, N))
    return out[0] if one else out


def adjoint_int32(W: np.ndarray, y: np.ndarray, n: int) -> np.ndarray:
    """Integer adjoint: (W^T)^{kron n} y mod 2^32 (real W, so ^H is ^T)."""
    return staged_int32(np.asarray(W).T, y, n)


def sylvester_hadamard(n: int) -> np.ndarray:
    """The natural-order (Sylvester) Walsh-Hadamard matrix with entries
    (-1)^{p . q}, where p . q is the bitwise dot product (popcount of p & q);
    §2.6, Hadamard reduction of the product formula (without the 1/sqrt(N))."""
    N = 1 << n
    H = np.empty((N, N), dtype=np.int64)
    for p in range(N):
        for q in range(N):
            H[p, q] = -1 if bin(p & q).count("1") % 2 else 1
    return H


# ---------------------------------------------------------------------------
# Applications used as next rows (§4.1.1 classical protocol, §4.3 filtering)
# ---------------------------------------------------------------------------
def natural_filter(W: np.ndarray, x: np.ndarray, n: int, cutoff: int):
    """Classical form of the natural-order filter of §4.3 (Alg. 3): transform,
    split the coefficients at natural index `cutoff` (k < c low, k >= c high),
    and transform each part back with G^dagger.  Returns (low, high)."""
    X = staged(W, x, n)
    idx = np.arange(X.shape[-1])
    lo = np.where(idx < cutoff, X, 0)
    hi = np.where(idx >= cutoff, X, 0)
    return adjoint(W, lo, n), adjoint(W, hi, n)


def topk_compress(W: np.ndarray, x: np.ndarray, n: int, k: int):
    """Classical state-transmission protocol of §4.1.1: transform, keep the k
    coefficients of largest magnitude (ties broken towards the lower index),
    reconstruct with G^dagger.  Returns (kept_indices ascending, kept values,
    reconstruction)."""
    X = np.asarray(staged(W, x, n))
    mag = np.abs(X)
    # stable order on (-|c|, index): the lower index wins a tie
    order = np.lexsort((np.arange(X.size), -mag))
    keep = np.sort(order[:k])
    Xk = np.zeros_like(X)
    Xk[keep] = X[keep]
    return keep, X[keep], adjoint(W, Xk, n)


def kept_energy(coeffs_kept: np.ndarray, coeffs_all: np.ndarray) -> float:
    """sum |kept|^2 / sum |all|^2 (the fidelity of the renormalised truncated
    state with the original, for a unitary transform; §4.1.5)."""
    return float(np.sum(np.abs(coeffs_kept) ** 2) / np.sum(np.abs(coeffs_all) ** 2))


def fidelity(psi: np.ndarray, phi: np.ndarray) -> float:
    """F = |<psi|phi>|^2 for normalised states (§4.1.5)."""
    psi = np.asarray(psi) / np.linalg.norm(psi)
    phi = np.asarray(phi) / np.linalg.norm(phi)
    return float(abs(np.vdot(psi, phi)) ** 2)
