"""Plain FP64 CPU reference for the FFT-accelerated CG homogenisation solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module: it exists so that the tests, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` can check the HIP library against
an implementation that is slow, obviously correct and independent of it.  It
shares no code with the GPU path.

The method is Zeman, Vondrejc, Novak, Marek, "Accelerating a FFT-based solver
for numerical homogenization of periodic media by conjugate gradients"
(J. Comput. Phys., 2010).  Every function below names the passage it follows.

Conventions (documented readings of the paper, see also the repository notes):

* A field with ``d`` components on an ``N_1 x ... x N_d`` grid is an array of
  shape ``(d, N_1, ..., N_d)``; array index ``j`` sits at coordinate
  ``x = j / N`` of the unit cell (a cyclic shift of the paper's centred node
  numbering, Sec. 2.2, Eq. (10)).
* Phases are isotropic, ``L(x) = lambda(x) I``, or symmetric tensors
  (``Medium``); the reference medium is ``L0 = l0 I`` (Sec. 3) or any
  symmetric positive definite ``d x d`` matrix (Sec. 2.1, Eq. (7)): every
  ``l0`` argument takes either form.
* The DFT is unnormalised forward, ``1/|N|`` inverse.  The ``|Y|^{-1/2}`` and
  ``|Y|^{1/2}`` factors of the Vandermonde matrices (Sec. 2.2, Eqs. (13)-(14))
  cancel inside the operator ``B`` of Eq. (16).
* Integer frequencies ``k`` of the set ``Z^N`` (Sec. 2.2, Eq. (9)) are exact
  for a cubic cell.  For even ``N_alpha`` the Green operator is set to zero on
  every mode with ``k_alpha = N_alpha / 2`` (the paper only uses odd grids;
  this reading keeps the discrete operator real).
* CG is the unpreconditioned Hestenes-Stiefel method cited in Sec. 3 as
  Saad's Algorithm 6.18, with Euclidean inner products over all ``d |N|``
  entries and ``x0 = e0``.  It stops when ``||r_m||_2 <= tol ||e0||_2`` (the
  relative residual; the paper's ``eta_r`` of Eq. (22) is reported beside it).
  For an anisotropic ``L0`` the system matrix is self-adjoint (on the
  fields the iterates live in) only in the energy product of the reference
  medium, ``<u, v>_L0 = sum_x u(x) . L0 . v(x)``; CG and the basic scheme
  then take that product and its norm.  For ``L0 = l0 I`` it is ``l0`` times
  the Euclidean one, so nothing changes.  BiCG, meant for non-symmetric
  systems, keeps the Euclidean product.
* The homogenised conductivity is ``L_eff E = <lambda e>``, the cell average
  of the current ``j = L e`` of Sec. 2.1, Eq. (1); the full tensor comes from
  ``d`` load cases.

Parity pins: every function here is checked by the ``not gpu`` tests against
values fixed by the mathematics (explicit Vandermonde matrices, a dense direct
solve, closed-form laminates, bounds, duality, an independent fixed-point
solver).  See ``tests/test_oracle_pins.py``.
"""

from __future__ import annotations

import math
import os

import numpy as np

try:  # scipy.fft keeps float32 in single precision and can use threads
    import scipy.fft as _sfft
except Exception:  # pragma: no cover - scipy is present in this image
    _sfft = None

__all__ = [
    "frequencies",
    "grid_frequencies",
    "wave_vectors",
    "Medium",
    "reference_matrix",
    "green_hat",
    "apply_B",
    "apply_A",
    "apply_BT",
    "apply_AT",
    "cg",
    "bicg",
    "pipelined_cg",
    "ffth",
    "dense_operator",
    "dense_solve",
    "leff",
    "homogenize",
    "eta_r",
    "eta_e",
    "eta_e_from_residual",
    "project_gradient",
    "optimal_reference",
    "mean_reference",
    "reference_omega",
    "voigt_reuss",
    "cg_rate_bound_iterations",
]

_WORKERS = int(os.environ.get("LSHOM_ORACLE_WORKERS", os.cpu_count() or 1))


def _fftn(a, axes):
    if _sfft is not None:
        return _sfft.fftn(a, axes=axes, workers=_WORKERS)
    return np.fft.fftn(a, axes=axes)


def _ifftn(a, axes):
    if _sfft is not None:
        return _sfft.ifftn(a, axes=axes, workers=_WORKERS)
    return np.fft.ifftn(a, axes=axes)


# ---------------------------------------------------------------------------
# Frequencies and the Green operator (Sec. 2.1, Eq. (7); Sec. 2.2, Eq. (9))
# ---------------------------------------------------------------------------

def frequencies(n: int) -> np.ndarray:
    """Integer frequencies of one axis, in DFT index order.

    The set ``Z^N = {k : -N/2 < k <= N/2}`` (Sec. 2.2, Eq. (9)); DFT index
    ``m`` carries frequency ``m`` if ``m <= N/2`` and ``m - N`` otherwise.
    """
    m = np.arange(n)
    return np.where(m <= n // 2, m, m - n).astype(np.float64)


def grid_frequencies(shape):
    """Per-axis integer frequency arrays broadcast over the grid ``shape``."""
    d = len(shape)
    out = []
    for a, n in enumerate(shape):
        k = frequencies(n)
        view = [1] * d
        view[a] = n
        out.append(np.broadcast_to(k.reshape(view), shape))
    return out


def _nyquist_mask(shape):
    """True on modes kept by the Green operator (all but k_alpha = N_alpha/2)."""
    keep = np.ones(shape, dtype=bool)
    for a, n in enumerate(shape):
        if n % 2 == 0:
            idx = [slice(None)] * len(shape)
            idx[a] = n // 2
            keep[tuple(idx)] = False
    return keep


def wave_vectors(shape, cell=None):
    """Wave vector components xi_alpha = k_alpha / Y_alpha on the DFT grid.

    The basis of Sec. 2.1, Eq. (6) has exp(i pi x_alpha k_alpha / Y_alpha) on
    the cell prod (-Y_alpha, Y_alpha): derivatives scale mode k by k / Y, so
    the Green operator of Eq. (7) for a non-cubic cell takes xi in place of
    the integer k (a common factor pi cancels in it).  ``cell`` holds the d
    side lengths (None: a cubic cell, xi = k)."""
    ks = grid_frequencies(shape)
    if cell is None:
        return ks
    return [k / float(c) for k, c in zip(ks, cell)]


def reference_matrix(l0, d):
    """The reference conductivity as ``(L0, iso)``.

    ``l0`` is a number (``L0 = l0 I``, the isotropic reference of Sec. 3) or
    a symmetric positive definite ``d x d`` matrix (the general ``L0`` of
    Sec. 2.1, Eqs. (3) and (7)).  A matrix equal to a multiple of ``I`` is
    returned as that number (``iso`` True), so both spellings of an
    isotropic reference give identical results."""
    if np.ndim(l0) == 0:
        return float(l0), True
    m = np.array(l0, dtype=np.float64)
    if m.shape != (d, d):
        raise ValueError(f"L0 must be a number or a {d} x {d} matrix")
    if not np.allclose(m, m.T, rtol=0.0, atol=1e-12 * np.abs(m).max()):
        raise ValueError("L0 must be symmetric")
    m = 0.5 * (m + m.T)
    if np.linalg.eigvalsh(m).min() <= 0.0:
        raise ValueError("L0 must be positive definite")
    if np.all(m == m[0, 0] * np.eye(d)):
        return float(m[0, 0]), True
    return m, False


def reference_scale(l0, d) -> float:
    """``l0`` of an isotropic reference, ``tr(L0) / d`` otherwise: the factor
    in front of the residual norm of Sec. 3, Eq. (22)."""
    L0, iso = reference_matrix(l0, d)
    return L0 if iso else float(np.trace(L0)) / d


def _quad(L0, xs):
    """``x . L0 . x`` at every grid point for the component arrays ``xs``."""
    d = len(xs)
    return sum(L0[a, b] * xs[a] * xs[b] for a in range(d) for b in range(d))


def _green_factors(shape, l0, cell=None):
    """Wave vectors and ``1 / (xi . L0 . xi)`` (zero where Gamma0 is 0)."""
    ks = wave_vectors(shape, cell)
    k2 = sum(k * k for k in ks)
    keep = _nyquist_mask(shape) & (k2 > 0)
    inv = np.zeros(shape)
    L0, iso = reference_matrix(l0, len(shape))
    q = L0 * k2 if iso else _quad(L0, ks)
    inv[keep] = 1.0 / q[keep]
    return ks, inv


def _energy_dot(l0, d):
    """Inner product of CG and of the basic scheme's test: Euclidean for an
    isotropic reference, ``sum_x u . L0 . v`` otherwise."""
    L0, iso = reference_matrix(l0, d)
    if iso:
        return _dot
    d = L0.shape[0]

    def dot(u, v):
        gram = u.reshape(d, -1) @ v.reshape(d, -1).T  # sum_x u_a(x) v_b(x)
        return float(np.sum(L0 * gram))
    return dot


class Medium:
    """A digital microstructure and its cell.

    ``lam`` is a scalar conductivity per node (shape ``N``: isotropic phases,
    Sec. 3) or a symmetric tensor per node (shape ``(d, d, *N)``: the
    second-order conductivity of Sec. 2.1, Eq. (1)); ``cell`` holds the d
    side lengths of the cell (None: cubic).  Functions of this module accept
    a Medium wherever they take ``lam``; a plain array is an isotropic medium
    on a cubic cell."""

    def __init__(self, lam, cell=None):
        lam = np.asarray(lam, dtype=np.float64)
        self.tensor = lam.ndim >= 4 and lam.shape[0] == lam.shape[1] == lam.ndim - 2
        self.lam = lam
        self.shape = lam.shape[2:] if self.tensor else lam.shape
        self.d = len(self.shape)
        self.cell = None if cell is None else tuple(float(c) for c in cell)
        if self.cell is not None and len(self.cell) != self.d:
            raise ValueError("cell needs one length per axis")

    def times(self, p, shift=0.0):
        """``(L - shift) p`` at every node (p: ``(d, *N)``); ``shift`` is a
        number (``shift I``) or a constant ``d x d`` matrix (``L - L0`` of
        Sec. 2.1, Eq. (3) for an anisotropic reference)."""
        if np.ndim(shift) == 2:
            m = np.asarray(shift, dtype=np.float64)
            return self.times(p) - np.einsum("ab,b...->a...", m, p)
        if self.tensor:
            out = np.einsum("ab...,b...->a...", self.lam, p)
            return out - shift * p if shift else out
        return (self.lam - shift)[None, ...] * p

    def eigen_range(self):
        """Smallest and largest eigenvalue of L over all nodes."""
        if not self.tensor:
            return float(self.lam.min()), float(self.lam.max())
        m = np.moveaxis(self.lam.reshape(self.d, self.d, -1), -1, 0)
        w = np.linalg.eigvalsh(m)
        return float(w.min()), float(w.max())


def _medium(lam):
    return lam if isinstance(lam, Medium) else Medium(lam)


def green_hat(shape, l0: float) -> np.ndarray:
    """Blocks of the reference Green operator on the DFT grid.

    ``G[alpha, beta][k] = k_alpha k_beta / (k . L0 . k)`` for ``k != 0`` and
    ``0`` at ``k = 0`` (Sec. 2.1, Eq. (7)), with ``L0 = l0 I`` or a general
    matrix ``l0``.  Returns an array of shape ``(d, d, *shape)``.
    """
    ks = grid_frequencies(shape)
    d = len(shape)
    k2 = sum(k * k for k in ks)
    keep = _nyquist_mask(shape) & (k2 > 0)
    inv = np.zeros(shape)
    L0, iso = reference_matrix(l0, d)
    q = L0 * k2 if iso else _quad(L0, ks)
    inv[keep] = 1.0 / q[keep]
    g = np.empty((d, d) + tuple(shape))
    for a in range(d):
        for b in range(d):
            g[a, b] = ks[a] * ks[b] * inv
    return g


# ---------------------------------------------------------------------------
# The operator of the collocation system (Sec. 2.2, Eqs. (15)-(17))
# ---------------------------------------------------------------------------

def apply_B(p: np.ndarray, lam, l0: float) -> np.ndarray:
    """``B p = F^{-1} Gamma0_hat F (dL p)`` with ``dL = L - L0``.

    Sec. 2.2, Eq. (16): polarisation by the blocks ``dL_ab`` (Eq. (3) and
    Eq. (17); diagonal in the nodes, full d x d for tensor phases), forward
    DFT of each component, the block-diagonal Green operator of Eq. (7),
    inverse DFT.  The result is real for real input.
    """
    med = _medium(lam)
    shape = med.shape
    d = len(shape)
    axes = tuple(range(1, d + 1))
    tau = med.times(p, reference_matrix(l0, d)[0])
    tau_hat = _fftn(tau, axes)
    ks, inv = _green_factors(shape, l0, med.cell)
    w_hat = np.zeros_like(tau_hat)
    for a in range(d):
        for b in range(d):
            # block (a, b) of Eq. (16): diagonal Gamma0_hat_ab times tau_hat_b
            w_hat[a] += (ks[a] * ks[b] * inv) * tau_hat[b]
    return _ifftn(w_hat, axes).real


def apply_A(p: np.ndarray, lam, l0: float) -> np.ndarray:
    """``(I + B) p``, the left-hand side of the collocation system, Eq. (15)."""
    return p + apply_B(p, lam, l0)


def apply_BT(p: np.ndarray, lam, l0: float) -> np.ndarray:
    """``B^T p = dL F^{-1} Gamma0_hat F p``: the factors of Eq. (16) in the
    other order (``dL`` is symmetric block-diagonal and ``F^{-1} Gamma0_hat
    F`` is a real symmetric matrix), the product BiCG needs besides ``B``
    (Sec. 2.3)."""
    med = _medium(lam)
    shape = med.shape
    d = len(shape)
    axes = tuple(range(1, d + 1))
    p_hat = _fftn(np.asarray(p, dtype=np.float64), axes)
    ks, inv = _green_factors(shape, l0, med.cell)
    w_hat = np.zeros_like(p_hat)
    for a in range(d):
        for b in range(d):
            w_hat[a] += (ks[a] * ks[b] * inv) * p_hat[b]
    return med.times(_ifftn(w_hat, axes).real, reference_matrix(l0, d)[0])


def apply_AT(p: np.ndarray, lam, l0: float) -> np.ndarray:
    """``(I + B)^T p``."""
    return p + apply_BT(p, lam, l0)


def _dot(u, v) -> float:
    return float(np.dot(u.ravel(), v.ravel()))


def _rhs(E, shape):
    E = np.asarray(E, dtype=np.float64)
    d = len(shape)
    if E.shape != (d,):
        raise ValueError(f"E must have {d} components")
    return np.broadcast_to(E.reshape((d,) + (1,) * d), (d,) + tuple(shape)).copy()


def optimal_reference(lam) -> float:
    """``l0 = (lambda_min + lambda_max) / 2``, Sec. 2.3, Eq. (19): the extreme
    eigenvalues of L over the cell."""
    lo, hi = _medium(lam).eigen_range()
    return 0.5 * (lo + hi)


def mean_reference(lam):
    """``L0 = <L>``, the cell average of the conductivity (a matrix; a number
    for isotropic phases).  In the spectral coordinate the diagonal of the
    operator K*LK (K: c -> i khat c) is ``khat . <L> . khat``, so this
    reference is the Fourier-space Jacobi preconditioner of CG in the energy
    product of L0 (Sec. 2.1, Eq. (7) with a general L0)."""
    med = _medium(lam)
    if not med.tensor:
        return float(np.mean(med.lam))
    return med.lam.reshape(med.d, med.d, -1).mean(axis=2)


def reference_omega(omega: float, rho: float) -> float:
    """``l0(omega) = 1 - omega + rho omega``, Sec. 3, Eq. (20)."""
    return 1.0 - omega + rho * omega


# ---------------------------------------------------------------------------
# Conjugate gradients (Sec. 2.3 and Sec. 3: Saad, Algorithm 6.18)
# ---------------------------------------------------------------------------

def cg(lam, l0, E, tol=1e-8, max_iter=10000, x0=None, n_iter=None,
       history=False, apply=None, norm="r", eta_history=False):
    """Solve ``(I + B) e = e0`` by Hestenes-Stiefel CG.

    Follows the CG method the paper applies to the collocation system
    (Sec. 2.3; Sec. 3 names it Saad's Algorithm 6.18):

    ``r0 = b - A x0``, ``p0 = r0``; per iteration ``q = A p``,
    ``alpha = (r, r) / (p, q)``, ``x += alpha p``, ``r -= alpha q``,
    ``beta = (r_new, r_new) / (r, r)``, ``p = r + beta p``.  The products
    are Euclidean for ``L0 = l0 I`` and the energy product of ``L0``
    otherwise (module notes), with the norm of the test and of ``eta_r``
    taken from the same product.

    The test ``||r|| <= tol ||b||`` is made before each iteration, so the
    returned iteration count is the number of operator applies in the loop.
    ``n_iter`` forces exactly that many iterations (used to compare with the
    GPU at an equal iteration count).  ``x0`` defaults to ``b``.

    ``norm="eta_e"`` replaces the test by the equilibrium criterion of
    Sec. 3, Eq. (21), ``eta_e(x_m) <= tol``, evaluated from its definition on
    the current iterate.  ``eta_history`` records ``(eta_r, eta_e)`` of every
    iterate ``x_0 .. x_m`` (``eta_r`` of Eq. (22) from the recursive residual).

    Returns a dict with the field ``e``, ``iterations``, ``rel_res`` (the
    recursive residual), ``converged``, ``breakdown`` and optionally the
    residual ``history`` and ``eta_history``.
    """
    if norm not in ("r", "eta_e"):
        raise ValueError("norm must be 'r' or 'eta_e'")
    lam = _medium(lam)
    shape = lam.shape
    A = apply if apply is not None else (lambda v: apply_A(v, lam, l0))
    dot = _energy_dot(l0, lam.d)
    lsc = reference_scale(l0, lam.d)
    b = _rhs(E, shape)
    bnorm = math.sqrt(dot(b, b))
    if bnorm == 0.0:
        return dict(e=np.zeros_like(b), iterations=0, rel_res=0.0,
                    converged=True, breakdown=False, r=np.zeros_like(b),
                    history=[0.0])
    x = b.copy() if x0 is None else np.array(x0, dtype=np.float64, copy=True)
    r = b - A(x)
    p = r.copy()
    rr = dot(r, r)
    hist = [math.sqrt(rr) / bnorm]
    etas = []

    def stop_test():
        eta_e_x = eta_e(lam, x) if (norm == "eta_e" or eta_history) else None
        if eta_history:
            etas.append((lsc * math.sqrt(rr) / bnorm, eta_e_x))
        if norm == "eta_e":
            return eta_e_x <= tol
        return math.sqrt(rr) <= tol * bnorm

    m = 0
    limit = max_iter if n_iter is None else n_iter
    converged = False
    breakdown = False
    while True:
        ok = stop_test()
        if n_iter is None and ok:
            converged = True
            break
        if m >= limit:
            break
        q = A(p)
        pq = dot(p, q)
        if not (pq > 0.0) or not math.isfinite(pq):
            breakdown = True
            break
        alpha = rr / pq
        x += alpha * p
        r -= alpha * q
        rr_new = dot(r, r)
        beta = rr_new / rr
        p = r + beta * p
        rr = rr_new
        m += 1
        hist.append(math.sqrt(rr) / bnorm)
    if n_iter is not None:
        converged = ok
    out = dict(e=x, iterations=m, rel_res=math.sqrt(rr) / bnorm,
               converged=converged, breakdown=breakdown, r=r)
    if history:
        out["history"] = hist
    if eta_history:
        out["eta_history"] = etas
    return out


def pipelined_cg(lam, l0, E, tol=1e-8, max_iter=10000, n_iter=None):
    """CG with one reduction phase per iteration (Ghysels and Vanroose,
    Parallel Computing 40 (2014), the pipelined CG without preconditioner).

    The paper's outlook asks for faster variants of its CG; this one gives
    the same iterates in exact arithmetic while both inner products of an
    iteration are formed together and may overlap the operator apply.  With
    ``w = A r`` carried as a vector: ``gamma = (r, r)``, ``delta = (w, r)``,
    ``n = A w``; ``beta = gamma / gamma_prev`` and ``alpha = gamma / (delta -
    beta gamma / alpha_prev)`` (``beta = 0``, ``alpha = gamma / delta`` at the
    start); ``z = n + beta z``, ``s = w + beta s``, ``p = r + beta p``,
    ``x += alpha p``, ``r -= alpha s``, ``w -= alpha z``.  Products, norms and
    the stopping test are those of ``cg`` (which it must reproduce); ``n_iter``
    forces that many iterations.
    """
    lam = _medium(lam)
    dot = _energy_dot(l0, lam.d)
    b = _rhs(E, lam.shape)
    bnorm = math.sqrt(dot(b, b))
    if bnorm == 0.0:
        return dict(e=np.zeros_like(b), iterations=0, rel_res=0.0, converged=True, breakdown=False)

    def A(v):
        return apply_A(v, lam, l0)

    x = b.copy()
    r = b - A(x)
    w = A(r)
    z = np.zeros_like(b)
    s = np.zeros_like(b)
    p = np.zeros_like(b)
    gamma_prev = alpha_prev = None
    m = 0
    limit = max_iter if n_iter is None else n_iter
    converged = breakdown = False
    while True:
        gamma = dot(r, r)
        delta = dot(w, r)
        if n_iter is None and math.sqrt(gamma) <= tol * bnorm:
            converged = True
            break
        if m >= limit:
            break
        n = A(w)
        if m == 0:
            beta, alpha = 0.0, gamma / delta
        else:
            beta = gamma / gamma_prev
            alpha = gamma / (delta - beta * gamma / alpha_prev)
        if not (alpha > 0.0) or not math.isfinite(alpha):
            breakdown = True
            break
        z = n + beta * z
        s = w + beta * s
        p = r + beta * p
        x += alpha * p
        r -= alpha * s
        w -= alpha * z
        gamma_prev, alpha_prev = gamma, alpha
        m += 1
    rel = math.sqrt(dot(r, r)) / bnorm
    if n_iter is not None:
        converged = rel <= tol
    return dict(e=x, iterations=m, rel_res=rel, converged=converged, breakdown=breakdown)


def bicg(lam, l0, E, tol=1e-8, max_iter=10000, n_iter=None):
    """Solve ``(I + B) e = e0`` by the biconjugate gradient method.

    Sec. 2.3 proposes it beside CG and Sec. 3 names Saad's Algorithm 7.3:
    ``r0 = b - A x0``, shadow residual ``r0* = r0``, ``p0 = r0``,
    ``p0* = r0*``; per iteration ``alpha = (r, r*) / (A p, p*)``,
    ``x += alpha p``, ``r -= alpha A p``, ``r* -= alpha A^T p*``,
    ``beta = (r_new, r*_new) / (r, r*)``, ``p = r + beta p``,
    ``p* = r* + beta p*``.  The test ``||r|| <= tol ||b||`` precedes each
    iteration (as in ``cg``); ``n_iter`` forces that many iterations.
    Products and norms are Euclidean for every reference medium.
    """
    lam = _medium(lam)
    shape = lam.shape
    b = _rhs(E, shape)
    bnorm = math.sqrt(_dot(b, b))
    x = b.copy()
    if bnorm == 0.0:
        return dict(e=np.zeros_like(b), iterations=0, rel_res=0.0, converged=True, breakdown=False)
    r = b - apply_A(x, lam, l0)
    rs = r.copy()
    p = r.copy()
    ps = rs.copy()
    rho = _dot(r, rs)
    m = 0
    limit = max_iter if n_iter is None else n_iter
    converged = breakdown = False
    while True:
        rn = math.sqrt(_dot(r, r))
        if n_iter is None and rn <= tol * bnorm:
            converged = True
            break
        if m >= limit:
            break
        ap = apply_A(p, lam, l0)
        sigma = _dot(ap, ps)
        if sigma == 0.0 or not math.isfinite(sigma):
            breakdown = True
            break
        alpha = rho / sigma
        x += alpha * p
        r -= alpha * ap
        rs -= alpha * apply_AT(ps, lam, l0)
        rho_new = _dot(r, rs)
        beta = rho_new / rho
        p = r + beta * p
        ps = rs + beta * ps
        rho = rho_new
        m += 1
    rel = math.sqrt(_dot(r, r)) / bnorm
    if n_iter is not None:
        converged = rel <= tol
    return dict(e=x, iterations=m, rel_res=rel, converged=converged, breakdown=breakdown)


def true_residual(lam, l0, E, e, euclidean=False) -> float:
    """``||b - (I + B) e|| / ||b||`` evaluated afresh (Eq. (15)), in the norm
    of ``cg`` (the energy norm of an anisotropic ``L0``; Euclidean with
    ``euclidean=True``, the norm of ``bicg``)."""
    med = _medium(lam)
    dot = _dot if euclidean else _energy_dot(l0, med.d)
    b = _rhs(E, med.shape)
    bn = math.sqrt(dot(b, b))
    res = b - apply_A(e, lam, l0)
    return math.sqrt(dot(res, res)) / bn if bn > 0 else 0.0


# ---------------------------------------------------------------------------
# The basic Moulinec-Suquet scheme (Sec. 2.3, Eq. (18))
# ---------------------------------------------------------------------------

def ffth(lam, l0, E, tol=1e-8, max_iter=100000, norm="r", eta_history=False):
    """Neumann-series iterate ``e^(m) = sum_{j<=m} (-B)^j e0``.

    Sec. 2.3, Eq. (18), evaluated as ``e^(m+1) = e0 - B e^(m)``.  Stops after
    the apply in which the test on ``e^(m)`` holds and returns ``e^(m+1)``:
    ``||e^(m+1) - e^(m)|| <= tol ||e0||`` (``eta_r / l0`` of Eq. (22)), or with
    ``norm="eta_e"`` ``eta_e(e^(m)) <= tol`` (Eq. (21)); the step norm is
    that of ``cg`` (energy norm of an anisotropic ``L0``).  ``eta_history``
    records ``(eta_r, eta_e)`` of ``e^(0) .. e^(m)``, where the residual of
    ``e^(m)`` is the step ``e^(m+1) - e^(m)``.
    """
    if norm not in ("r", "eta_e"):
        raise ValueError("norm must be 'r' or 'eta_e'")
    lam = _medium(lam)
    dot = _energy_dot(l0, lam.d)
    lsc = reference_scale(l0, lam.d)
    b = _rhs(E, lam.shape)
    bnorm = math.sqrt(dot(b, b))
    e = b.copy()
    etas = []
    for m in range(1, max_iter + 1):
        e_new = b - apply_B(e, lam, l0)
        diff = e_new - e
        step = math.sqrt(dot(diff, diff))
        eta_e_m = eta_e(lam, e) if (norm == "eta_e" or eta_history) else None
        if eta_history:
            etas.append((lsc * step / bnorm, eta_e_m))
        e = e_new
        ok = eta_e_m <= tol if norm == "eta_e" else step <= tol * bnorm
        if ok:
            out = dict(e=e, iterations=m, converged=True)
            break
    else:
        out = dict(e=e, iterations=max_iter, converged=False)
    if eta_history:
        out["eta_history"] = etas
    return out


# ---------------------------------------------------------------------------
# Dense matrices of the collocation system (Sec. 2.2, Eqs. (13)-(17))
# ---------------------------------------------------------------------------

def _centred_indices(n):
    """The centred index set ``Z^N`` of one axis (Sec. 2.2, Eq. (9))."""
    return np.array([k for k in range(-(n // 2), n // 2 + 1)
                     if -n / 2 < k <= n / 2], dtype=np.int64)


def dense_operator(lam, l0, cell_measure=1.0):
    """The matrix ``I + B`` built entry by entry from Sec. 2.2.

    Nodes and frequencies are both numbered by the centred set ``Z^N``
    (Eq. (9)) exactly as in the paper; ``F`` and ``F^{-1}`` are the
    Vandermonde matrices of Eqs. (13)-(14) including the ``|Y|`` factors,
    ``Gamma0_hat`` and ``dL`` are the diagonal blocks of Eq. (17), and ``B``
    is the product of Eq. (16).  Only for tiny grids.

    Returns ``(M, order)`` where ``M`` acts on vectors stacked as
    ``[component][node]`` with nodes in the centred order, and ``order`` maps
    each centred node to its flat array index (``j = k mod N``).
    """
    med = _medium(lam)
    shape = med.shape
    d = len(shape)
    idx = [_centred_indices(n) for n in shape]
    grids = np.meshgrid(*idx, indexing="ij")
    K = np.stack([g.ravel() for g in grids], axis=1)  # (|N|, d) centred ints
    nn = K.shape[0]
    Nvec = np.array(shape, dtype=np.float64)
    phase = -2j * np.pi * ((K[:, None, :] * K[None, :, :]) / Nvec).sum(axis=2)
    F = cell_measure ** -0.5 * np.exp(phase)
    Finv = cell_measure ** 0.5 / nn * np.exp(-phase)
    flat = np.ravel_multi_index(tuple((K % np.array(shape)).T), shape)
    # node blocks dL_ab = L_ab - L0_ab (Eqs. (3), (17)): diagonal matrices
    L0m, iso = reference_matrix(l0, d)
    L0 = L0m * np.eye(d) if iso else L0m
    if med.tensor:
        dl = [[med.lam[a, b].ravel()[flat] - L0[a, b] for b in range(d)] for a in range(d)]
    else:
        diag = med.lam.ravel()[flat]
        dl = [[(diag if a == b else np.zeros(nn)) - L0[a, b] for b in range(d)] for a in range(d)]
    # Green operator blocks (Eq. (7)) at xi = k / Y
    Y = np.ones(d) if med.cell is None else np.array(med.cell)
    X = K.astype(np.float64) / Y[None, :]
    k2 = (X ** 2).sum(axis=1)
    keep = k2 > 0
    for a, n in enumerate(shape):
        if n % 2 == 0:
            keep &= K[:, a] != n // 2
    xLx = np.einsum("na,ab,nb->n", X, L0, X)
    G = [[np.where(keep, X[:, a] * X[:, b] / np.where(keep, xLx, 1.0), 0.0) for b in range(d)]
         for a in range(d)]
    B = np.zeros((d * nn, d * nn), dtype=np.complex128)
    for a in range(d):
        for c in range(d):
            # block (a, c) of Eq. (16): sum_b F^-1 G_ab F dL_bc
            blk = np.zeros((nn, nn), dtype=np.complex128)
            for b in range(d):
                blk += Finv @ (G[a][b][:, None] * (F * dl[b][c][None, :]))
            B[a * nn:(a + 1) * nn, c * nn:(c + 1) * nn] = blk
    M = np.eye(d * nn) + B
    return M, flat


def dense_solve(lam, l0, E, cell_measure=1.0):
    """Direct solution of Eq. (15) with the dense matrix of ``dense_operator``."""
    shape = _medium(lam).shape
    d = len(shape)
    M, flat = dense_operator(lam, l0, cell_measure)
    nn = flat.size
    rhs = np.concatenate([np.full(nn, float(E[a])) for a in range(d)]).astype(np.complex128)
    sol = np.linalg.solve(M, rhs)
    e = np.zeros((d, int(np.prod(shape))))
    for a in range(d):
        e[a, flat] = sol[a * nn:(a + 1) * nn].real
    return e.reshape((d,) + shape), float(np.abs(sol.imag).max())


# ---------------------------------------------------------------------------
# Outputs and norms
# ---------------------------------------------------------------------------

def leff(lam, e) -> np.ndarray:
    """``L_eff E = <lambda e>``: cell average of the current ``j = L e``.

    Sec. 2.1, Eqs. (1)-(2): ``j = L e`` with ``<e> = e0``; the macroscopic
    current is the average of ``j``.  Returns ``d`` numbers (one column of the
    effective tensor for the load case that produced ``e``).
    """
    med = _medium(lam)
    j = med.times(e)
    return np.array([float(np.mean(j[a])) for a in range(med.d)])


def homogenize(lam, l0=None, tol=1e-10, max_iter=10000):
    """Full effective tensor from the ``d`` load cases ``E = e_beta``."""
    lam = _medium(lam)
    d = lam.d
    l0 = optimal_reference(lam) if l0 is None else l0
    L = np.zeros((d, d))
    iters = []
    for b in range(d):
        E = np.zeros(d)
        E[b] = 1.0
        res = cg(lam, l0, E, tol=tol, max_iter=max_iter)
        L[:, b] = leff(lam, res["e"])
        iters.append(res["iterations"])
    return L, iters


def eta_r(r, l0, E, shape) -> float:
    """Residual norm ``l0 ||r|| / ||e0||`` (Sec. 3, Eq. (22)); for an
    anisotropic ``L0``, ``tr(L0) / d`` times the energy-norm ratio."""
    d = len(shape)
    dot = _energy_dot(l0, d)
    b = _rhs(E, shape)
    return reference_scale(l0, d) * math.sqrt(dot(r, r)) / math.sqrt(dot(b, b))


def eta_e(lam, e) -> float:
    """Equilibrium norm of Sec. 3, Eq. (21).

    ``eta_e^2 = sum_k |k . j_hat(k)|^2 / |j_hat(0)|^2`` with ``j = lambda e``
    and integer frequencies; the ratio does not depend on DFT scaling.
    """
    med = _medium(lam)
    d = med.d
    axes = tuple(range(1, d + 1))
    j_hat = _fftn(med.times(e), axes)
    ks = wave_vectors(med.shape, med.cell)
    div = sum(ks[a] * j_hat[a] for a in range(d))
    num = float(np.sum(np.abs(div) ** 2))
    zero = (0,) * d
    den = float(sum(abs(j_hat[a][zero]) ** 2 for a in range(d)))
    return math.sqrt(num / den)


def eta_e_from_residual(lam, l0, E, e) -> float:
    """``eta_e`` through the residual of an admissible field ``e``.

    With ``r = e0 - (I + B) e`` and ``j = lambda e``: for ``k != 0``,
    ``k . j_hat = k . tau_hat + l0 k . e_hat`` (``tau = (lambda - l0) e``) and
    ``k . r_hat = -k . e_hat - k . tau_hat / l0`` (Sec. 2.2, Eqs. (15)-(17)),
    so ``k . j_hat = -l0 k . r_hat``; ``r_hat(k)`` is parallel to ``k`` for
    the gradient fields of Sec. 2.1, hence ``|k . r_hat| = |k| |r_hat|``.
    For a general ``L0`` the same steps give ``r_hat = -k (k . j_hat) /
    (k . L0 . k)``, so ``|k . j_hat| = |r_hat| (k . L0 . k) / |k|``.
    Valid for odd grids (no Nyquist modes, where the Green operator is zero).
    """
    med = _medium(lam)
    d = med.d
    axes = tuple(range(1, d + 1))
    r = _rhs(E, med.shape) - apply_A(e, med, l0)
    r_hat = _fftn(r, axes)
    ks = wave_vectors(med.shape, med.cell)
    k2 = sum(ks[a].astype(np.float64) ** 2 for a in range(d))
    r2 = sum(np.abs(r_hat[a]) ** 2 for a in range(d))
    L0, iso = reference_matrix(l0, d)
    if iso:
        num = float(np.sum(k2 * r2))
    else:
        q = _quad(L0, ks)
        nz = k2 > 0
        num = float(np.sum(q[nz] ** 2 / k2[nz] * r2[nz]))
    j_hat = _fftn(med.times(e), axes)
    zero = (0,) * d
    den = float(sum(abs(j_hat[a][zero]) ** 2 for a in range(d)))
    return (L0 if iso else 1.0) * math.sqrt(num / den)


def project_gradient(v: np.ndarray) -> np.ndarray:
    """Orthogonal projection onto zero-mean curl-free grid fields.

    ``P v = F^{-1}[ k (k . v_hat) / |k|^2 ]`` with ``P v_hat(0) = 0``: the
    Green operator of Eq. (7) with ``L0 = I``.  Used to make a warm start
    admissible, ``x0 = E + P(x_pred)``.
    """
    shape = v.shape[1:]
    d = len(shape)
    axes = tuple(range(1, d + 1))
    ks, inv = _green_factors(shape, 1.0)
    v_hat = _fftn(v, axes)
    s = sum(ks[b] * v_hat[b] for b in range(d)) * inv
    w_hat = np.stack([ks[a] * s for a in range(d)])
    return _ifftn(w_hat, axes).real


def voigt_reuss(lam):
    """Arithmetic (Voigt) and harmonic (Reuss) means of the nodal values."""
    lam = np.asarray(lam, dtype=np.float64)
    return float(np.mean(lam)), float(1.0 / np.mean(1.0 / lam))


def cg_rate_bound_iterations(rho: float, tol: float) -> int:
    """Iteration bound from the CG rate of Sec. 3.2, Eq. (23).

    ``||r_m|| <= 2 sqrt(kappa) gamma^m ||r_0||`` with
    ``gamma = (sqrt(rho) - 1) / (sqrt(rho) + 1)`` and ``kappa <= rho`` on the
    subspace CG works in; returns the smallest ``m`` that guarantees
    ``||r_m|| <= tol ||r_0||``.
    """
    g = (math.sqrt(rho) - 1.0) / (math.sqrt(rho) + 1.0)
    if g <= 0.0:
        return 1
    return int(math.ceil(math.log(tol / (2.0 * math.sqrt(rho))) / math.log(g)))
