"""FP64 CPU oracle for the point-process GLM log-likelihood and its gradient.

TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
bench's CPU-baseline leg may import this module; the library never does.
It shares no code with the GPU path.

What it computes (Zaytsev, Morrison, Deger, "Reconstruction of recurrent
synaptic connectivity of thousands of neurons from simulated spiking
activity"):

* Sec. 2.1, Eq. (1)-(2): L = sum_i L_i,
  L_i = sum_k log lambda_i(t_{i,k}) - integral lambda_i dt.
* Sec. 2.2, Eq. (3) and (5) with delta_u = 1: U_i = J_i0 + sum_j J_ij (h * s_j),
  h(t) = H(t) exp(-t/tau), lambda_i = exp(U_i).  J_i0 is called mu_i here.
* Sec. 2.3.3, Eq. (11)-(12): dL_i/dJ_ij = sum_k v_ij(t_{i,k}) - integral
  lambda_i v_ij dt, with v_ij = h * s_j and v_i0 = 1 (so dL_i/dmu_i = q_i -
  integral lambda_i dt).

Grid form (the method evaluated on a uniform grid of B bins of width dt,
covering [0, B dt)):

* s_i[t] = number of spikes of neuron i in bin t.
* trace x_j[t] = sum_{t' < t} a^(t-t'-1) s_j[t'], a = exp(-dt/tau); i.e.
  x_j[0] = 0, x_j[t] = a x_j[t-1] + s_j[t-1].  A spike acts on later bins only,
  with weight 1 in the next bin (the peak amplitude, as h(0) = 1).  This is the
  grid counterpart of the recurrence Eq. (13).
* U_i[t] = mu_i + sum_j J_ij x_j[t], lambda_i[t] = exp(U_i[t]) in 1/s.
* L_i = sum_t s_i[t] U_i[t] - dt sum_t lambda_i[t].  (The constant
  sum_t s_i[t] log dt that a binned likelihood would add is excluded.)
* dL/dJ_ij = sum_t (s_i[t] - dt lambda_i[t]) x_j[t],
  dL/dmu_i = q_i - dt sum_t lambda_i[t].
* dL/dtau = sum_{t,i} (s_i[t] - dt lambda_i[t]) sum_j J_ij y_j[t] with
  y_j = d x_j / d tau, y_j[0] = 0, y_j[t] = a y_j[t-1] + (dt/tau^2) a x_j[t-1]
  (the time constant is not part of theta_i, Sec. 2.2, so this gradient is
  taken separately).

Continuous-time form (tiny inputs only, used to pin the grid form): the
closed-form integral Eq. (9)-(10) with the exponential integral Ei (proof in
App. B), the gradient integral Eq. (14), and the same quantities by adaptive
quadrature.

Fits: exact per-row Newton (Hessian Eq. (18), App. A) for small problems,
scipy L-BFGS-B (the optimiser family of Sec. 2.6.3) on the joint vector for
larger ones, stopping on the fractional change of L (Sec. 2.6.3).

Classification: 1-D k-means with k = 3 (Sec. 3.3 / App. C.2), MER over the
off-diagonal pairs, the confusion bookkeeping of Tables 2, 3, 5, 6, and the
chance level MER_0 of Eq. (20).

Every function is plain FP64 NumPy/SciPy; nothing is blocked or fused beyond
time-chunking (a memory bound that does not change any value beyond rounding).
"""
from __future__ import annotations

import math
from typing import Dict, List, Optional, Sequence

import numpy as np
import scipy.integrate
import scipy.optimize
import scipy.signal
import scipy.sparse
import scipy.special

DEFAULT_CHUNK = 65536


# --------------------------------------------------------------------- data

def decay(dt: float, tau: float) -> float:
    """a = exp(-dt/tau): the kernel h decays by this factor per bin."""
    return math.exp(-dt / tau)


def spike_matrix(bins: np.ndarray, neurons: np.ndarray, N: int, B: int) -> scipy.sparse.csr_matrix:
    """S[t, i] = s_i[t], the spike count of neuron i in bin t (CSR, float64)."""
    bins = np.asarray(bins, dtype=np.int64)
    neurons = np.asarray(neurons, dtype=np.int64)
    if bins.size and (bins.min() < 0 or bins.max() >= B):
        raise ValueError("spike bin outside [0, B)")
    if neurons.size and (neurons.min() < 0 or neurons.max() >= N):
        raise ValueError("spike neuron outside [0, N)")
    data = np.ones(bins.shape[0], dtype=np.float64)
    S = scipy.sparse.coo_matrix((data, (bins, neurons)), shape=(B, N)).tocsr()
    S.sum_duplicates()
    return S


def spike_counts(neurons: np.ndarray, N: int) -> np.ndarray:
    """q_i: number of spikes of neuron i (Sec. 2.1)."""
    return np.bincount(np.asarray(neurons, dtype=np.int64), minlength=N).astype(np.int64)


# -------------------------------------------------------------------- trace

def trace_recursive(S: np.ndarray, a: float) -> np.ndarray:
    """x[0] = 0, x[t] = a x[t-1] + s[t-1]  (grid form of Eq. (13)); loop over t."""
    S = np.asarray(S, dtype=np.float64)
    X = np.zeros_like(S)
    for t in range(1, S.shape[0]):
        X[t] = a * X[t - 1] + S[t - 1]
    return X


def trace_direct(S: np.ndarray, a: float) -> np.ndarray:
    """x[t] = sum_{t' < t} a^(t-t'-1) s[t']  (the convolution h * s_j of Eq. (3)
    sampled on the grid); brute force, O(B^2)."""
    S = np.asarray(S, dtype=np.float64)
    B = S.shape[0]
    X = np.zeros_like(S)
    for t in range(B):
        for tp in range(t):
            X[t] += a ** (t - tp - 1) * S[tp]
    return X


def trace_rows(S: np.ndarray, a: float, x0: np.ndarray, out: Optional[np.ndarray] = None) -> np.ndarray:
    """The recursion x[t] = a x[t-1] + s[t-1] over the rows of a chunk, started
    from x[0] = x0 (the trace carried in from earlier bins)."""
    S = np.asarray(S, dtype=np.float64)
    X = np.empty_like(S) if out is None else out[: S.shape[0]]
    X[0] = x0
    for t in range(1, S.shape[0]):
        np.multiply(X[t - 1], a, out=X[t])
        X[t] += S[t - 1]
    return X


def trace_lfilter(S: np.ndarray, a: float, x0: Optional[np.ndarray] = None) -> np.ndarray:
    """The same trace as the IIR filter y[t] = a y[t-1] + s[t-1]
    (scipy.signal.lfilter with b = [0, 1], a = [1, -a]).  x0 is the trace value
    at the first row (the carry from earlier bins); it decays as a^t."""
    S = np.asarray(S, dtype=np.float64)
    X = scipy.signal.lfilter([0.0, 1.0], [1.0, -a], S, axis=0)
    if x0 is not None:
        X = X + np.power(a, np.arange(S.shape[0], dtype=np.float64))[:, None] * x0[None, :]
    return X


def tau_trace_recursive(S: np.ndarray, a: float, dt: float, tau: float):
    """(x, y) with y = dx/dtau: y[0] = 0, y[t] = a y[t-1] + (dt/tau^2) a x[t-1]."""
    S = np.asarray(S, dtype=np.float64)
    X = np.zeros_like(S)
    Y = np.zeros_like(S)
    c = dt / (tau * tau)
    for t in range(1, S.shape[0]):
        X[t] = a * X[t - 1] + S[t - 1]
        Y[t] = a * Y[t - 1] + c * a * X[t - 1]
    return X, Y


def tau_trace_direct(S: np.ndarray, a: float, dt: float, tau: float) -> np.ndarray:
    """y[t] = sum_{t'<t} (t-t'-1) a^(t-t'-1) (dt/tau^2) s[t'], the derivative of
    the direct sum with respect to tau (da/dtau = a dt / tau^2)."""
    S = np.asarray(S, dtype=np.float64)
    B = S.shape[0]
    Y = np.zeros_like(S)
    c = dt / (tau * tau)
    for t in range(B):
        for tp in range(t):
            m = t - tp - 1
            Y[t] += m * a ** m * c * S[tp]
    return Y


# ------------------------------------------------- likelihood and gradient

def _colsum(M: np.ndarray) -> np.ndarray:
    """Column sums as a two-level blocked sum: blocks of 256 rows, then the
    block sums (rounding error bounded by ~(256 + rows/256) ulp per column)."""
    M = np.asarray(M, dtype=np.float64)
    L = M.shape[0]
    nb = -(-L // 256)
    if nb * 256 != L:
        M = np.concatenate([M, np.zeros((nb * 256 - L,) + M.shape[1:])], axis=0)
    return M.reshape(nb, 256, *M.shape[1:]).sum(axis=1).sum(axis=0)


def loglik(bins, neurons, N: int, B: int, dt: float, tau: float, J: np.ndarray,
           mu: np.ndarray, want_grad: bool = True, want_tau: bool = False,
           chunk: int = DEFAULT_CHUNK, bin_range: Optional[Sequence[int]] = None,
           rows: Optional[Sequence[int]] = None) -> Dict:
    """Grid log-likelihood (Eq. (2)/(7)) and gradient (Eq. (12)) in FP64.

    J[i, j] is the weight from presynaptic j to postsynaptic i, mu[i] = J_i0.
    Returns a dict with
      ll       total log-likelihood (float)
      ll_rows  L_i per neuron [N]
      spike_term, integral_term  the two parts of Eq. (7) per neuron [N]
      gJ [N, N], gmu [N]  (if want_grad)
      gtau (float)        (if want_tau)
      q [N]               spike counts
    bin_range = (b0, b1) restricts every sum over t to bins b0 <= t < b1 (the
    trace still sees every spike before b1); used for bounded timing samples.
    rows = list of postsynaptic neurons restricts the output to those rows
    (L is separable over rows, Sec. 2.2): ll_rows, spike_term, integral_term,
    gmu and q then have len(rows) entries and gJ has len(rows) rows; ll and
    gtau are the sums over those rows only.
    The time axis is processed in chunks of `chunk` bins with the trace value
    carried exactly across chunk boundaries.
    """
    J = np.asarray(J, dtype=np.float64)
    mu = np.asarray(mu, dtype=np.float64)
    S = spike_matrix(bins, neurons, N, B)
    a = decay(dt, tau)
    c_tau = dt / (tau * tau)
    b0, b1 = (0, B) if bin_range is None else (int(bin_range[0]), int(bin_range[1]))
    rsel = np.arange(N) if rows is None else np.asarray(rows, dtype=np.int64)
    pos = np.full(N, -1, dtype=np.int64)
    pos[rsel] = np.arange(rsel.shape[0])
    J = J[rsel]
    mu = mu[rsel]
    R_n = rsel.shape[0]
    spike_parts: List[np.ndarray] = []
    integ_parts: List[np.ndarray] = []
    gJ = np.zeros((R_n, N)) if want_grad else None
    lam_parts: List[np.ndarray] = []
    gtau_parts: List[float] = []
    x_carry = np.zeros(N)
    y_carry = np.zeros(N)
    # carry the trace through the skipped prefix [0, b0) without summing
    if b0 > 0:
        for t0 in range(0, b0, chunk):
            t1 = min(t0 + chunk, b0)
            Sc = S[t0:t1].toarray()
            Xc = trace_rows(Sc, a, x_carry)
            if want_tau:
                Yc = trace_rows(c_tau * a * Xc, a, y_carry)
                y_carry = a * Yc[-1] + c_tau * a * Xc[-1]
            x_carry = a * Xc[-1] + Sc[-1]
    JT = np.ascontiguousarray(J.T)
    nrow = min(chunk, max(b1 - b0, 1))
    Sbuf = np.zeros((nrow, N))
    Xbuf = np.empty((nrow, N))
    for t0 in range(b0, b1, chunk):
        t1 = min(t0 + chunk, b1)
        Ssp = S[t0:t1]
        coo = Ssp.tocoo()
        Sc = Sbuf[: t1 - t0]
        Sc.fill(0.0)
        Sc[coo.row, coo.col] = coo.data
        Xc = trace_rows(Sc, a, x_carry, out=Xbuf)
        x_carry = a * Xc[-1] + Sc[-1]
        U = Xc @ JT
        U += mu[None, :]
        # sum over the spikes of U at their bins (the first term of Eq. (7))
        keep = pos[coo.col] >= 0
        spike_parts.append(np.bincount(pos[coo.col[keep]],
                                       weights=coo.data[keep] * U[coo.row[keep], pos[coo.col[keep]]],
                                       minlength=R_n))
        lam = np.exp(U, out=U)
        lam_sum = _colsum(lam)
        integ_parts.append(dt * lam_sum)
        lam_parts.append(lam_sum)
        R = lam
        R *= -dt
        R += Sc if rows is None else Sc[:, rsel]  # s - dt lambda
        if want_grad:
            gJ += R.T @ Xc
        if want_tau:
            Yc = trace_rows(c_tau * a * Xc, a, y_carry)
            V = Yc @ JT
            gtau_parts.append(float(np.sum(_colsum(R * V))))
            y_carry = a * Yc[-1] + c_tau * a * Xc[-1]
    spike_term = np.array([math.fsum(p[i] for p in spike_parts) for i in range(R_n)])
    integral_term = np.array([math.fsum(p[i] for p in integ_parts) for i in range(R_n)])
    ll_rows = spike_term - integral_term
    q = np.asarray(S[b0:b1].sum(axis=0)).ravel()[rsel]
    out = dict(ll=math.fsum(ll_rows), ll_rows=ll_rows, spike_term=spike_term,
               integral_term=integral_term, q=q)
    if want_grad:
        lam_total = np.array([math.fsum(p[i] for p in lam_parts) for i in range(R_n)])
        out["gJ"] = gJ
        out["gmu"] = q - dt * lam_total
    if want_tau:
        out["gtau"] = math.fsum(gtau_parts)
    return out


def loglik_delayed(bins, neurons, N: int, B: int, dt: float, tau: float, J: np.ndarray,
                   mu: np.ndarray, d: int, d_self: int) -> Dict:
    """Grid L_i and gradient with transmission delays (Sec. 2.4, Eq. (15)) in
    FP64, dense (small inputs): row i sees every presynaptic trace x_j with
    j != i delayed by d bins and its own x_i by d_self bins, while its spike
    terms stay at the recorded bins:
        U_i[t] = mu_i + sum_{j != i} J_ij x_j[t - d] + J_ii x_i[t - d_self],
        L_i = sum_t s_i[t] U_i[t] - dt sum_t exp(U_i[t]),
        dL/dJ_ij = sum_t (s_i[t] - dt lambda_i[t]) x_j[t - D_ij],
    with x_j[t] = 0 for t <= 0 (the trace of reading R1)."""
    S = spike_matrix(bins, neurons, N, B).toarray()
    X = trace_lfilter(S, decay(dt, tau))

    def delayed(k):
        out = np.zeros_like(X)
        if k < B:
            out[k:] = X[:B - k]
        return out

    Xd, Xs = delayed(d), delayed(d_self)
    off = J * (1.0 - np.eye(N))
    U = mu[None, :] + Xd @ off.T + Xs * np.diag(J)[None, :]
    lam = np.exp(U)
    R = S - dt * lam
    ll_rows = (S * U).sum(axis=0) - dt * lam.sum(axis=0)
    gJ = R.T @ Xd
    gJ[np.arange(N), np.arange(N)] = (R * Xs).sum(axis=0)
    return dict(ll_rows=ll_rows, ll=float(math.fsum(ll_rows)), gJ=gJ, gmu=R.sum(axis=0))


def spike_term_matrix(bins, neurons, N: int, B: int, dt: float, tau: float,
                      chunk: int = DEFAULT_CHUNK) -> np.ndarray:
    """partial^Sigma_ij = sum_t s_i[t] x_j[t] (Eq. (12)); parameter-free; computed once per tau (Sec. 2.3.3)."""
    S = spike_matrix(bins, neurons, N, B)
    a = decay(dt, tau)
    D = np.zeros((N, N))
    x_carry = np.zeros(N)
    for t0 in range(0, B, chunk):
        t1 = min(t0 + chunk, B)
        Sc = S[t0:t1].toarray()
        Xc = trace_lfilter(Sc, a, x_carry)
        D += Sc.T @ Xc
        x_carry = a * Xc[-1] + Sc[-1]
    return D


def dense_trace(bins, neurons, N: int, B: int, dt: float, tau: float) -> np.ndarray:
    """The whole trace matrix X [B, N] (small problems only)."""
    S = spike_matrix(bins, neurons, N, B).toarray()
    return trace_lfilter(S, decay(dt, tau))


# ---------------------------------------------------------------- fitting

def _row_objective(A: np.ndarray, s: np.ndarray, dt: float, theta: np.ndarray):
    """L_i, gradient and Hessian for one row with design A = [1, X] (Eq. (18))."""
    U = A @ theta
    lam = np.exp(U)
    L = math.fsum(s * U) - dt * math.fsum(lam)
    g = A.T @ (s - dt * lam)
    H = -dt * (A.T * lam[None, :]) @ A
    return L, g, H


def newton_fit(bins, neurons, N: int, B: int, dt: float, tau: float,
               J0: Optional[np.ndarray] = None, mu0: Optional[np.ndarray] = None,
               rows: Optional[Sequence[int]] = None, fit_J: bool = True,
               max_iter: int = 100, eta_tol: float = 1e-15):
    """Exact per-row Newton ascent with backtracking (small problems only).

    Each row theta_i = (mu_i, J_i1..J_iN) is a separate concave problem
    (Sec. 2.2, App. A).  Iterates until the fractional change of L_i is below
    eta_tol (Sec. 2.6.3) and the Newton decrement vanishes.  fit_J=False keeps
    J fixed at J0 and fits mu only.
    Returns (J, mu, info) with info['iters'] per row."""
    S = spike_matrix(bins, neurons, N, B).toarray()
    X = trace_lfilter(S, decay(dt, tau))
    J = np.zeros((N, N)) if J0 is None else np.array(J0, dtype=np.float64)
    mu = np.zeros(N) if mu0 is None else np.array(mu0, dtype=np.float64)
    rows = range(N) if rows is None else rows
    iters = {}
    for i in rows:
        s = S[:, i]
        if fit_J:
            A = np.concatenate([np.ones((B, 1)), X], axis=1)
            theta = np.concatenate([[mu[i]], J[i]])
        else:
            A = np.ones((B, 1))
            theta = np.array([mu[i]])
            s_off = X @ J[i]
        def obj(th):
            if fit_J:
                return _row_objective(A, s, dt, th)
            U = th[0] + s_off
            lam = np.exp(U)
            L = math.fsum(s * U) - dt * math.fsum(lam)
            return L, np.array([s.sum() - dt * lam.sum()]), np.array([[-dt * lam.sum()]])
        L, g, H = obj(theta)
        k = 0
        for k in range(1, max_iter + 1):
            step = np.linalg.solve(H, -g)  # ascent direction (H negative definite)
            decrement = float(g @ step)  # Newton decrement g^T (-H)^-1 g >= 0
            t = 1.0
            while True:
                Ln, gn, Hn = obj(theta + t * step)
                if np.isfinite(Ln) and Ln >= L + 1e-4 * t * float(g @ step):
                    break
                t *= 0.5
                if t < 1e-12:
                    Ln, gn, Hn = L, g, H
                    break
            eta = abs(Ln - L) / max(abs(Ln), 1e-300)
            theta = theta + t * step
            L, g, H = Ln, gn, Hn
            if eta <= eta_tol or decrement <= 1e-13 * max(abs(L), 1.0):
                break
        iters[i] = k
        mu[i] = theta[0]
        if fit_J:
            J[i] = theta[1:]
    return J, mu, dict(iters=iters)


def _trace_chunks(S, a: float, chunk: int):
    """The trace of a recording chunk by chunk, (b0, X_chunk) with the value at
    each chunk's first bin carried over from the chunk before."""
    N = S.shape[1]
    B = S.shape[0]
    x0 = np.zeros(N)
    for b0 in range(0, B, chunk):
        b1 = min(B, b0 + chunk)
        Sc = S[b0:b1].toarray().astype(np.float64)
        X = trace_lfilter(Sc, a, x0)
        # the trace at bin b1: one more step of the recursion from the chunk's last row
        x0 = a * X[-1] + Sc[-1]
        yield b0, X


def _rows_pass(chunks, s_rows: Dict[int, np.ndarray], dt: float, thetas: Dict[int, np.ndarray],
               hessian: bool):
    """One pass over the time axis for the rows in `thetas` (row -> (mu_i, J_i)):
    L_i and, if `hessian`, the gradient and the Hessian of Eq. (18), each summed
    chunk by chunk.  `chunks` yields (b0, trace chunk); s_rows[i] is row i's
    spike counts per bin."""
    parts = {i: [] for i in thetas}
    P = None
    g = H = None
    for b0, X in chunks:
        if P is None:
            P = X.shape[1] + 1
            g = {i: np.zeros(P) for i in thetas} if hessian else None
            H = {i: np.zeros((P, P)) for i in thetas} if hessian else None
        b1 = b0 + X.shape[0]
        for i, th in thetas.items():
            s = s_rows[i][b0:b1]
            U = th[0] + X @ th[1:]
            lam = np.exp(U)
            parts[i].append(float(np.sum(s * U)) - dt * float(np.sum(lam)))
            if hessian:
                r = s - dt * lam
                g[i][0] += r.sum()
                g[i][1:] += X.T @ r
                w = dt * lam
                Xw = X.T @ w
                H[i][0, 0] -= w.sum()
                H[i][0, 1:] -= Xw
                H[i][1:, 0] -= Xw
                H[i][1:, 1:] -= (X * w[:, None]).T @ X
    L = {i: math.fsum(v) for i, v in parts.items()}
    return L, g, H


def newton_rows(bins, neurons, N: int, B: int, dt: float, tau: float, rows: Sequence[int],
                max_iter: int = 60, eta_tol: float = 1e-15, chunk: int = DEFAULT_CHUNK,
                log=None, cache_bytes: float = 40e9):
    """Exact per-row Newton ascent for the rows `rows` of a recording too long
    for one dense trace matrix: L is separable over rows (Sec. 2.2) and each
    row's problem is concave (App. A), so each row's maximiser is found on its
    own with the Hessian of Eq. (18), summed over time chunks.  Start:
    J_i = 0 and mu_i = log(q_i / T) (the maximiser at J_i = 0).  A step is the
    Newton step scaled by t = 1, 1/2, 1/4, ... until the Armijo condition
    holds; the trial point's gradient and Hessian are taken in the same pass as
    its L.  A row stops when the fractional change of L_i is below eta_tol
    (Sec. 2.6.3) or its Newton decrement vanishes.  The trace chunks are kept
    in memory when they take at most cache_bytes.
    Returns dict(row -> dict(mu, J, ll, iters, decrement, se)); se holds the
    standard errors sqrt(diag(-H^-1)) of (mu_i, J_i) at the result (the
    curvature of Eq. (18), the resolution the data allow)."""
    S = spike_matrix(bins, neurons, N, B)
    a = decay(dt, tau)
    q = spike_counts(neurons, N)
    Sc = S.tocsc()
    s_rows = {int(i): Sc[:, int(i)].toarray().ravel().astype(np.float64) for i in rows}
    if 8.0 * N * B <= cache_bytes:
        cached = list(_trace_chunks(S, a, chunk))
        chunks = lambda: iter(cached)  # noqa: E731
    else:
        chunks = lambda: _trace_chunks(S, a, chunk)  # noqa: E731
    th = {int(i): np.concatenate([[math.log(q[i] / (B * dt))], np.zeros(N)]) for i in rows}
    L, g, H = _rows_pass(chunks(), s_rows, dt, th, True)
    out = {}
    active = set(th)
    for k in range(1, max_iter + 1):
        if not active:
            break
        step = {i: np.linalg.solve(H[i], -g[i]) for i in active}
        dec = {i: float(g[i] @ step[i]) for i in active}
        t = {i: 1.0 for i in active}
        L_old = {i: L[i] for i in active}
        pending = set(active)
        while pending:
            trial = {i: th[i] + t[i] * step[i] for i in pending}
            Lt, gt, Ht = _rows_pass(chunks(), s_rows, dt, trial, True)
            for i in list(pending):
                if np.isfinite(Lt[i]) and Lt[i] >= L[i] + 1e-4 * t[i] * dec[i]:
                    th[i], L[i], g[i], H[i] = trial[i], Lt[i], gt[i], Ht[i]
                    pending.discard(i)
                else:
                    t[i] *= 0.5
                    if t[i] < 1e-12:
                        pending.discard(i)  # no ascent left: stay
        for i in list(active):
            eta = abs(L[i] - L_old[i]) / max(abs(L[i]), 1e-300)
            if log is not None:
                log(f"row {i} iter {k}: L {L[i]!r} eta {eta:.3e} decrement {dec[i]:.3e} step {t[i]}")
            if eta <= eta_tol or dec[i] <= 1e-13 * max(abs(L[i]), 1.0):
                out[i] = dict(mu=float(th[i][0]), J=th[i][1:].copy(), ll=L[i], iters=k, decrement=dec[i],
                              se=np.sqrt(np.diag(np.linalg.inv(-H[i]))))
                active.discard(i)
    for i in active:  # iteration cap
        out[i] = dict(mu=float(th[i][0]), J=th[i][1:].copy(), ll=L[i], iters=max_iter, decrement=float("nan"),
                      se=np.sqrt(np.diag(np.linalg.inv(-H[i]))))
    return out


def _trace_chunks_loop(S, a: float, chunk: int):
    """The trace chunk by chunk by the recursion itself (trace_rows), carried
    across chunk boundaries; (b0, X_chunk)."""
    N = S.shape[1]
    B = S.shape[0]
    x0 = np.zeros(N)
    for b0 in range(0, B, chunk):
        b1 = min(B, b0 + chunk)
        Sc = S[b0:b1].toarray().astype(np.float64)
        X = trace_rows(Sc, a, x0)
        x0 = a * X[-1] + Sc[-1]
        yield b0, X


def newton_rows_sub(bins, neurons, N: int, B: int, dt: float, tau: float, rows: Sequence[int],
                    hess_stride: int = 8, refresh: int = 4, max_iter: int = 200,
                    step_tol: float = 1e-10, chunk: int = DEFAULT_CHUNK, log=None):
    """Maximiser of L_i for many rows of a long recording, with the Newton
    matrix taken on a subsample of the time axis.

    The target is the same as newton_rows': the unique point where the exact
    gradient of the concave row problem vanishes (Sec. 2.2 separability,
    App. A concavity).  L_i and its gradient (Eq. (7), (12)) are summed over
    every bin at every iterate.  Only the matrix that scales the step differs:
    the Hessian of Eq. (18) accumulated over every hess_stride-th time chunk
    and scaled by B / (bins in those chunks), recomputed at the first
    `refresh` iterates and then kept.  A fixed point of
    theta <- theta - H_sub^-1 g is a zero of the exact g whatever H_sub is (as
    long as it is negative definite), so the approximation slows the last
    iterations from quadratic to linear convergence and leaves the result
    unchanged.  Steps are backtracked (t = 1, 1/2, ...) to the Armijo
    condition on the exact L_i, except once the decrement g^T (-H_sub)^-1 g
    is below 1e-12 |L_i|: there L_i is quadratic in the error and its change
    is below its own rounding, and the full step (a contraction of the error
    in the local quadratic model) is taken on the gradient's evidence alone.
    Linear convergence makes a small change of L_i (Sec. 2.6.3's test) a weak
    sign of a small error, so a row stops when its accepted step moves no
    entry by more than step_tol.  All rows are evaluated in one pass per
    iterate (X Theta^T and X^T R as matrix products over the rows).
    Returns dict(row -> dict(mu, J, ll, iters, decrement, max_abs_grad, se));
    se = sqrt(diag(-H_sub^-1)) at the last refresh, an estimate of the
    standard errors (a scale for distances, not a reference value)."""
    rows = [int(i) for i in rows]
    R_n = len(rows)
    S = spike_matrix(bins, neurons, N, B)
    a = decay(dt, tau)
    q = spike_counts(neurons, N)
    Sr = S.tocsc()[:, rows].toarray().astype(np.float64)  # [B, R] spike counts of the rows
    chunk_starts = list(range(0, B, chunk))
    sampled = [k for k in range(len(chunk_starts)) if k % hess_stride == 0]
    n_sampled = sum(min(B, chunk_starts[k] + chunk) - chunk_starts[k] for k in sampled)
    scale = B / n_sampled

    def rows_pass(Th, hess_rows):
        """L [R], gradient [R, N+1] and the subsampled Hessians [R, N+1, N+1]
        of the rows in hess_rows at the parameters Th [R, N+1]."""
        want_H = bool(hess_rows)
        parts = [[] for _ in range(R_n)]
        g = np.zeros((R_n, N + 1))
        H = np.zeros((R_n, N + 1, N + 1)) if want_H else None
        for k, (b0, X) in enumerate(_trace_chunks_loop(S, a, chunk)):
            b1 = b0 + X.shape[0]
            s = Sr[b0:b1]
            U = X @ Th[:, 1:].T + Th[None, :, 0]  # [K, R]
            lam = np.exp(U)
            for r in range(R_n):
                parts[r].append(math.fsum(s[:, r] * U[:, r]) - dt * math.fsum(lam[:, r]))
            Rres = s - dt * lam
            g[:, 0] += Rres.sum(axis=0)
            g[:, 1:] += (X.T @ Rres).T
            if want_H and k in sampled:
                for r in hess_rows:
                    w = dt * lam[:, r]
                    Xw = X.T @ w
                    H[r, 0, 0] -= w.sum()
                    H[r, 0, 1:] -= Xw
                    H[r, 1:, 0] -= Xw
                    Xs = X * np.sqrt(w)[:, None]
                    H[r, 1:, 1:] -= Xs.T @ Xs  # sum_t w_t x_t x_t^T
        if want_H:
            H *= scale
        return np.array([math.fsum(p) for p in parts]), g, H

    Th = np.zeros((R_n, N + 1))
    Th[:, 0] = [math.log(q[i] / (B * dt)) for i in rows]
    L, g, H = rows_pass(Th, list(range(R_n)))
    active = list(range(R_n))
    out = {}
    for k in range(1, max_iter + 1):
        if not active:
            break
        step = {r: np.linalg.solve(H[r], -g[r]) for r in active}
        dec = {r: float(g[r] @ step[r]) for r in active}
        t = {r: 1.0 for r in active}
        L_old = L.copy()
        pending = list(active)
        want_H = k < refresh
        while pending:
            Tt = Th.copy()
            for r in pending:
                Tt[r] = Th[r] + t[r] * step[r]
            Lt, gt, Ht = rows_pass(Tt, pending if want_H else [])
            still = []
            for r in pending:
                floor = dec[r] <= 1e-12 * max(abs(L[r]), 1.0)
                if np.isfinite(Lt[r]) and (floor or Lt[r] >= L[r] + 1e-4 * t[r] * dec[r]):
                    Th[r], L[r], g[r] = Tt[r], Lt[r], gt[r]
                    if want_H:
                        H[r] = Ht[r]
                else:
                    t[r] *= 0.5
                    if t[r] >= 1e-12:
                        still.append(r)
                    else:
                        t[r] = 0.0
            pending = still
        for r in list(active):
            eta = abs(L[r] - L_old[r]) / max(abs(L[r]), 1e-300)
            moved = t[r] * float(np.abs(step[r]).max())
            if log is not None:
                log(f"row {rows[r]} iter {k}: L {L[r]!r} eta {eta:.3e} decrement {dec[r]:.3e} "
                    f"step {t[r]} moved {moved:.3e}")
            if moved <= step_tol:
                out[rows[r]] = dict(mu=float(Th[r, 0]), J=Th[r, 1:].copy(), ll=float(L[r]), iters=k,
                                    decrement=dec[r], max_abs_grad=float(np.abs(g[r]).max()),
                                    se=np.sqrt(np.diag(np.linalg.inv(-H[r]))))
                active.remove(r)
    for r in active:  # iteration cap
        out[rows[r]] = dict(mu=float(Th[r, 0]), J=Th[r, 1:].copy(), ll=float(L[r]), iters=max_iter,
                            decrement=float("nan"), max_abs_grad=float(np.abs(g[r]).max()),
                            se=np.sqrt(np.diag(np.linalg.inv(-H[r]))))
    return out


def lbfgs_fit(bins, neurons, N: int, B: int, dt: float, tau: float,
              J0: Optional[np.ndarray] = None, mu0: Optional[np.ndarray] = None,
              ftol: float = 1e-15, gtol: float = 1e-10, maxiter: int = 5000,
              chunk: int = DEFAULT_CHUNK):
    """scipy L-BFGS-B on the joint vector (mu, J) maximising L (Sec. 2.6.3)."""
    J = np.zeros((N, N)) if J0 is None else np.array(J0, dtype=np.float64)
    mu = np.zeros(N) if mu0 is None else np.array(mu0, dtype=np.float64)
    theta0 = np.concatenate([mu, J.ravel()])

    def f(theta):
        r = loglik(bins, neurons, N, B, dt, tau, theta[N:].reshape(N, N), theta[:N],
                   want_grad=True, chunk=chunk)
        return -r["ll"], -np.concatenate([r["gmu"], r["gJ"].ravel()])

    res = scipy.optimize.minimize(f, theta0, jac=True, method="L-BFGS-B",
                                  options=dict(ftol=ftol, gtol=gtol, maxiter=maxiter,
                                               maxcor=10))
    return res.x[N:].reshape(N, N), res.x[:N], res


# ------------------------------- penalty and bound constraints (Sec. 2.5, 2.6.3)

def l1_eps_penalty(J: np.ndarray, alpha: float, eps: float):
    """The smooth epsilon-l1 penalty of Eq. (16)-(17) per row,
    alpha * sum_{j != i} sqrt(J_ij^2 + eps), and its derivative with respect to
    J_ij, alpha * J_ij / sqrt(J_ij^2 + eps) (zero on the diagonal: the
    self-connection is not penalised)."""
    J = np.asarray(J, dtype=np.float64)
    off = ~np.eye(J.shape[0], J.shape[1], dtype=bool)
    r = np.sqrt(J * J + eps)
    pen = alpha * np.where(off, r, 0.0).sum(axis=1)
    dpen = alpha * np.where(off, J / r, 0.0)
    return pen, dpen


def penalized_fit(bins, neurons, N: int, B: int, dt: float, tau: float, alpha: float = 0.0,
                  eps: float = 1e-8, j_max: Optional[float] = None,
                  rate_min: Optional[float] = None, rate_max: Optional[float] = None,
                  ftol: float = 1e-15, gtol: float = 1e-12, maxiter: int = 20000):
    """Maximise L_i - alpha sum_{j != i} sqrt(J_ij^2 + eps) for every row i
    (Eq. (16)-(17)) subject to |J_ij| <= j_max and rate_min <= e^{mu_i} <=
    rate_max (the bounds of Sec. 2.6.3), by scipy's L-BFGS-B, the bounded
    quasi-Newton method the paper used.  The objective is separable over rows,
    so each row is its own problem.  Returns (J, mu, results)."""
    S = spike_matrix(bins, neurons, N, B).toarray()
    X = trace_lfilter(S, decay(dt, tau))
    A = np.concatenate([np.ones((B, 1)), X], axis=1)
    lo_mu = math.log(rate_min) if rate_min else None
    hi_mu = math.log(rate_max) if rate_max else None
    bounds = [(lo_mu, hi_mu)] + [(-j_max, j_max) if j_max else (None, None)] * N
    J = np.zeros((N, N))
    mu = np.zeros(N)
    results = []
    for i in range(N):
        s = S[:, i]

        def f(th):
            U = A @ th
            lam = np.exp(U)
            L = float(s @ U) - dt * float(lam.sum())
            g = A.T @ (s - dt * lam)
            Jr = th[1:]
            r = np.sqrt(Jr * Jr + eps)
            pen = alpha * (r.sum() - r[i])
            d = alpha * Jr / r
            d[i] = 0.0
            return -(L - pen), -(g - np.concatenate([[0.0], d]))

        th0 = np.zeros(N + 1)
        if lo_mu is not None or hi_mu is not None:
            th0[0] = min(max(0.0, lo_mu if lo_mu is not None else -np.inf),
                         hi_mu if hi_mu is not None else np.inf)
        res = scipy.optimize.minimize(f, th0, jac=True, method="L-BFGS-B", bounds=bounds,
                                      options=dict(ftol=ftol, gtol=gtol, maxiter=maxiter, maxcor=10))
        mu[i] = res.x[0]
        J[i] = res.x[1:]
        results.append(res)
    return J, mu, results


# ------------------------------------------- continuous time (tiny inputs)

def _ei_diff(D: float, xi: float) -> float:
    """Ei(D) - Ei(D xi) for 0 < xi < 1 and D of either sign.  For small |D| the
    two Ei values nearly cancel; then use Ei(x) = gamma + ln|x| + sum_n x^n/(n n!),
    whose difference is ln(1/xi) + sum_n D^n (1 - xi^n)/(n n!)."""
    if D == 0.0:
        return -math.log(xi)
    if abs(D) < 1e-2:
        acc = -math.log(xi)
        term = 1.0
        for n in range(1, 30):
            term *= D / n  # D^n / n!
            acc += term * (1.0 - xi ** n) / n
        return acc
    return float(scipy.special.expi(D) - scipy.special.expi(D * xi))


def _events(spike_times: Sequence[np.ndarray]):
    ev = []
    for j, ts in enumerate(spike_times):
        for t in np.asarray(ts, dtype=np.float64):
            ev.append((float(t), j))
    ev.sort()
    return ev


def continuous_ll(spike_times: Sequence[np.ndarray], T0: float, T1: float, tau: float,
                  J: np.ndarray, mu: np.ndarray, method: str = "ei") -> np.ndarray:
    """Continuous-time L_i for every neuron (Eq. (2), (7)).

    The potential follows the key recurrence Eq. (8) between the network's
    events t_1..t_q (with t_0 = T0, t_{q+1} = T1).  The integral term is the
    closed form Eq. (10) ("ei") or adaptive quadrature of Eq. (9) per interval
    ("quad").  The intensity at a spike of neuron i is the left limit (the
    spike does not act on its own intensity at its own time)."""
    N = len(spike_times)
    ev = _events(spike_times)
    times = [T0] + [t for t, _ in ev] + [T1]
    out = np.zeros(N)
    for i in range(N):
        c = math.exp(mu[i])
        D = 0.0  # U - J_i0 right after the current event
        spike_sum = []
        integ = []
        for k in range(len(times) - 1):
            tk, tk1 = times[k], times[k + 1]
            if k >= 1:
                j = ev[k - 1][1]
                # value just before this event (left limit) is D (already decayed)
                if j == i:
                    spike_sum.append(mu[i] + D)
                D += J[i, j]
            dtk = tk1 - tk
            xi = math.exp(-dtk / tau)
            if method == "ei":
                integ.append(c * tau * _ei_diff(D, xi))
            else:
                Dk = D
                val, _ = scipy.integrate.quad(lambda t: c * math.exp(Dk * math.exp(-(t - tk) / tau)),
                                              tk, tk1, epsabs=0.0, epsrel=1e-13, limit=200)
                integ.append(val)
            D *= xi
        out[i] = math.fsum(spike_sum) - math.fsum(integ)
    return out


def continuous_grad_integral(spike_times: Sequence[np.ndarray], T0: float, T1: float,
                             tau: float, J: np.ndarray, mu: np.ndarray, i: int,
                             method: str = "closed") -> np.ndarray:
    """partial^int_ij = integral lambda_i v_ij dt for all j (Eq. (12)), by the
    closed form Eq. (14) ("closed") or by quadrature ("quad")."""
    N = len(spike_times)
    ev = _events(spike_times)
    times = [T0] + [t for t, _ in ev] + [T1]
    c = math.exp(mu[i])
    D = 0.0
    v = np.zeros(N)
    parts = [[] for _ in range(N)]
    for k in range(len(times) - 1):
        tk, tk1 = times[k], times[k + 1]
        if k >= 1:
            j = ev[k - 1][1]
            D += J[i, j]
            v[j] += 1.0
        xi = math.exp(-(tk1 - tk) / tau)
        for j in range(N):
            if v[j] == 0.0:
                continue
            if method == "closed":
                if abs(D) < 1e-8:
                    f = (1.0 - xi) + D * (1.0 - xi * xi) / 2.0
                else:
                    f = (math.exp(D) - math.exp(D * xi)) / D
                parts[j].append(c * v[j] * tau * f)
            else:
                Dk, vk = D, v[j]
                val, _ = scipy.integrate.quad(
                    lambda t: c * math.exp(Dk * math.exp(-(t - tk) / tau)) * vk * math.exp(-(t - tk) / tau),
                    tk, tk1, epsabs=0.0, epsrel=1e-13, limit=200)
                parts[j].append(val)
        D *= xi
        v *= xi
    return np.array([math.fsum(p) for p in parts])


def _ei_diff_rows(D: np.ndarray, xi: float) -> np.ndarray:
    """_ei_diff for a vector of D at one xi: the series where |D| < 1e-2, the
    library exponential integral elsewhere."""
    out = np.empty_like(D)
    small = np.abs(D) < 1e-2
    for k in np.flatnonzero(small):
        out[k] = _ei_diff(float(D[k]), xi)
    big = ~small
    out[big] = scipy.special.expi(D[big]) - scipy.special.expi(D[big] * xi)
    return out


def continuous_eval(spike_times: Sequence[np.ndarray], T0: float, T1: float, tau: float,
                    J: np.ndarray, mu: np.ndarray) -> Dict[str, np.ndarray]:
    """Continuous-time L_i, dL/dJ_ij and dL/dmu_i of every neuron in one pass
    over the network's events (Eq. (7)-(8), (10), (12), (14)).

    v holds v_j right after the current event; over the interval that follows
    (length Delta, xi = e^{-Delta/tau}) neuron i has U_i = mu_i + D_i e^{-s/tau}
    with D = J v, whose integrals are tau e^{mu_i} [Ei(D_i) - Ei(D_i xi)]
    (Eq. (10)) and, against v_j e^{-s/tau}, tau e^{mu_i} v_j (e^{D_i} - e^{D_i xi}) / D_i
    (Eq. (14)).  At an event of neuron i its spike term takes the left limit
    U_i(t-) = mu_i + J_i . v and the trace v(t-) (Eq. (12)); the event's own
    jump comes after.  Equal times are taken in (time, neuron) order."""
    N = len(spike_times)
    ev = _events(spike_times)
    times = [T0] + [t for t, _ in ev] + [T1]
    c = np.exp(mu)
    v = np.zeros(N)
    spike = np.zeros(N)
    dsig = np.zeros((N, N))
    integ = np.zeros(N)
    G = np.zeros((N, N))
    q = np.zeros(N)
    for k in range(len(times) - 1):
        if k >= 1:
            j = ev[k - 1][1]
            spike[j] += mu[j] + J[j] @ v
            dsig[j] += v
            q[j] += 1
            v[j] += 1.0
        delta = (times[k + 1] - times[k]) / tau
        if delta > 0:
            xi = math.exp(-delta)
            D = J @ v
            integ += c * tau * _ei_diff_rows(D, xi)
            H = np.where(np.abs(D) < 1e-8, (1.0 - xi) + D * (1.0 - xi * xi) / 2.0,
                         (np.exp(D) - np.exp(D * xi)) / np.where(D == 0.0, 1.0, D))
            G += np.outer(c * tau * H, v)
            v = v * xi
    return dict(ll_rows=spike - integ, ll=float(math.fsum(spike - integ)), gJ=dsig - G, gmu=q - integ)


def _ei_diff_vec(D: np.ndarray, xi: np.ndarray) -> np.ndarray:
    """_ei_diff elementwise over arrays D and xi (0 < xi <= 1): the same
    three branches (D = 0; the series for |D| < 1e-2; the library Ei)."""
    D = np.asarray(D, dtype=np.float64)
    xi = np.broadcast_to(np.asarray(xi, dtype=np.float64), D.shape)
    out = np.empty_like(D)
    zero = D == 0.0
    out[zero] = -np.log(xi[zero])
    small = (np.abs(D) < 1e-2) & ~zero
    Ds, xs = D[small], xi[small]
    acc = -np.log(xs)
    term = np.ones_like(Ds)
    for n in range(1, 30):
        term = term * Ds / n  # D^n / n!
        acc = acc + term * (1.0 - xs ** n) / n
    out[small] = acc
    big = ~(zero | small)
    out[big] = scipy.special.expi(D[big]) - scipy.special.expi(D[big] * xi[big])
    return out


def continuous_eval_rows(times: np.ndarray, neurons: np.ndarray, N: int, T0: float, T1: float,
                         tau: float, J: np.ndarray, mu: np.ndarray, rows: Sequence[int],
                         chunk: int = DEFAULT_CHUNK) -> Dict[str, np.ndarray]:
    """continuous_eval for the postsynaptic rows `rows` only, over event lists
    too long for its per-event loop over all rows (Eq. (7)-(8), (10), (12),
    (14); L is separable over rows, Sec. 2.2).

    times, neurons: the network's events sorted by (time, neuron).  The same
    steps as continuous_eval, in the same order: the interval after event m
    (m = 0 is T0) starts with the trace v_m, which follows the recursion
    v_m = xi_{m-1} v_{m-1} + e_{j_m} (Eq. (8): decay over the interval before,
    then the jump of the event's neuron); at event m of a row's own neuron the
    spike term takes the left limit mu_i + J_i . (xi_{m-1} v_{m-1}); over the
    interval, D = J_i . v_m gives tau e^{mu_i} [Ei(D) - Ei(D xi)] (Eq. (10))
    and tau e^{mu_i} v_m (e^D - e^{D xi}) / D (Eq. (14)).  The trace vectors
    of a chunk of `chunk` intervals are formed by that recursion, one row per
    interval; the products with the rows' weights are matrix products.
    Returns dict(ll_rows, gJ [R, N], gmu, q) for the rows in the given order."""
    times = np.asarray(times, dtype=np.float64)
    neurons = np.asarray(neurons, dtype=np.int64)
    rows = np.asarray(rows, dtype=np.int64)
    R_n = rows.shape[0]
    pos = np.full(N, -1, dtype=np.int64)
    pos[rows] = np.arange(R_n)
    JR = np.asarray(J, dtype=np.float64)[rows]  # [R, N]
    muR = np.asarray(mu, dtype=np.float64)[rows]
    c = np.exp(muR)
    q_ev = times.shape[0]
    bounds = np.concatenate([[T0], times, [T1]])  # interval m is [bounds[m], bounds[m + 1])
    n_int = q_ev + 1
    spike_parts: List[np.ndarray] = []
    integ_parts: List[np.ndarray] = []
    G = np.zeros((R_n, N))
    dsig = np.zeros((R_n, N))
    q = np.zeros(R_n)
    v_prev = np.zeros(N)  # v_{m0 - 1} of the chunk's first interval m0
    xi_prev = 1.0         # and the decay over its interval
    for m0 in range(0, n_int, chunk):
        m1 = min(n_int, m0 + chunk)
        K = m1 - m0
        delta = (bounds[m0 + 1:m1 + 1] - bounds[m0:m1]) / tau
        xi = np.exp(-delta)
        V = np.empty((K, N))
        Vleft = np.empty((K, N))  # trace just before the chunk's events (left limits)
        for k in range(K):
            m = m0 + k
            if m == 0:
                Vleft[k] = 0.0
                V[k] = 0.0
                continue
            np.multiply(v_prev if k == 0 else V[k - 1], xi_prev if k == 0 else xi[k - 1], out=Vleft[k])
            V[k] = Vleft[k]
            V[k, neurons[m - 1]] += 1.0
        v_prev, xi_prev = V[-1].copy(), float(xi[-1])
        # spike terms of the rows' own events in this chunk
        ev = np.arange(max(m0, 1), m1)  # intervals that start at an event
        ev_neu = neurons[ev - 1]
        mine = pos[ev_neu] >= 0
        ev, ev_neu = ev[mine], ev_neu[mine]
        if ev.shape[0]:
            r_of = pos[ev_neu]
            Vl = Vleft[ev - m0]
            U_left = muR[r_of] + np.einsum("kn,kn->k", Vl, JR[r_of])
            spike_parts.append(np.bincount(r_of, weights=U_left, minlength=R_n))
            np.add.at(dsig, r_of, Vl)
            q += np.bincount(r_of, minlength=R_n)
        # integrals over the chunk's intervals of positive length
        live = delta > 0
        D = V[live] @ JR.T  # [K', R]
        xl = xi[live][:, None]
        integ_parts.append(tau * c * _ei_diff_vec(D, np.broadcast_to(xl, D.shape)).sum(axis=0))
        with np.errstate(divide="ignore", invalid="ignore"):
            H = np.where(np.abs(D) < 1e-8, (1.0 - xl) + D * (1.0 - xl * xl) / 2.0,
                         (np.exp(D) - np.exp(D * xl)) / np.where(D == 0.0, 1.0, D))
        G += (tau * c[None, :] * H).T @ V[live]
    spike = np.array([math.fsum(p[r] for p in spike_parts) for r in range(R_n)])
    integ = np.array([math.fsum(p[r] for p in integ_parts) for r in range(R_n)])
    ll_rows = spike - integ
    return dict(ll_rows=ll_rows, ll=float(math.fsum(ll_rows)), gJ=dsig - G, gmu=q - integ, q=q)


def grid_ll_from_times(spike_times: Sequence[np.ndarray], T: float, dt: float, tau: float,
                       J: np.ndarray, mu: np.ndarray) -> np.ndarray:
    """Bin continuous spike times on a grid of width dt and return the grid L_i."""
    N = len(spike_times)
    B = int(round(T / dt))
    bins, neu = [], []
    for j, ts in enumerate(spike_times):
        b = np.floor(np.asarray(ts) / dt).astype(np.int64)
        bins.append(b)
        neu.append(np.full(b.shape, j))
    bins = np.concatenate(bins)
    neu = np.concatenate(neu)
    return loglik(bins, neu, N, B, dt, tau, J, mu, want_grad=False)["ll_rows"]


# ------------------------------------------------------- classification

def kmeans3(values: np.ndarray, max_iter: int = 1000):
    """1-D Lloyd k-means with k = 3, initial centroids (min, 0, max), run to a
    fixed point.  Returns (labels, centroids); label 0 = lowest centroid
    (inhibitory), 1 = middle (unconnected), 2 = highest (excitatory)."""
    v = np.asarray(values, dtype=np.float64).ravel()
    c = np.array([v.min(), 0.0, v.max()])
    lab = None
    for _ in range(max_iter):
        d = np.abs(v[:, None] - c[None, :])
        new = np.argmin(d, axis=1)
        if lab is not None and np.array_equal(new, lab):
            break
        lab = new
        for k in range(3):
            if np.any(lab == k):
                c[k] = math.fsum(v[lab == k]) / int(np.sum(lab == k))
    order = np.argsort(c)
    remap = np.empty(3, dtype=np.int64)
    remap[order] = np.arange(3)
    return remap[lab], c[order]


def truth_classes(J_true: np.ndarray) -> np.ndarray:
    """0 = inhibitory (J < 0), 1 = none (J == 0), 2 = excitatory (J > 0)."""
    return np.where(J_true > 0, 2, np.where(J_true < 0, 0, 1))


def classify(J_hat: np.ndarray) -> np.ndarray:
    """k-means class of every off-diagonal entry (diagonal = -1: self-connections
    are treated separately, Sec. 3.1)."""
    N = J_hat.shape[0]
    off = ~np.eye(N, dtype=bool)
    lab, _ = kmeans3(J_hat[off])
    out = np.full((N, N), -1, dtype=np.int64)
    out[off] = lab
    return out


def mer(labels: np.ndarray, J_true: np.ndarray, is_exc: Optional[np.ndarray] = None) -> Dict:
    """Misclassification error rate over the off-diagonal pairs (Eq. (20)'s
    denominator N(N-1)) and over N^2 (the denominator of Tables 2-6), plus the
    per-class breakdown of the tables: each error is counted in the row of its
    true class (false negative) and of its assigned class (false positive);
    ND = errors violating Dale's law (presynaptic type vs assigned sign)."""
    N = J_true.shape[0]
    off = ~np.eye(N, dtype=bool)
    truth = truth_classes(J_true)
    wrong = off & (labels != truth)
    n_err = int(wrong.sum())
    rows = {}
    for k, name in ((2, "excitatory"), (0, "inhibitory"), (1, "unconnected")):
        fn = int((wrong & (truth == k)).sum())
        fp = int((wrong & (labels == k)).sum())
        row = dict(errors=fn + fp, fp=fp, fn=fn)
        if is_exc is not None and k != 1:
            pre_exc = np.broadcast_to(np.asarray(is_exc, dtype=bool)[None, :], (N, N))
            dale = wrong & (labels == k) & ((pre_exc & (k == 0)) | (~pre_exc & (k == 2)))
            row["nd"] = int(dale.sum())
        rows[name] = row
    total_rows = sum(r["errors"] for r in rows.values())
    return dict(errors=n_err, mer=n_err / (N * (N - 1)), mer_n2=n_err / (N * N),
                rows=rows, half_row_sum=total_rows // 2)


def mer0(p: float, f_e: float) -> float:
    """Chance-level MER of a random classifier that keeps p, f_e, f_i (Eq. (20))."""
    f_i = 1.0 - f_e
    return p * (2.0 - p * (1.0 + f_e * f_e + f_i * f_i))


def mer0_counts(p: float, f_e: float, N: int) -> float:
    """Eq. (20) from its three expected error counts n_e, n_i, n_n (App. C.1)."""
    f_i = 1.0 - f_e
    n_e = p * (f_e * N) * (N - 1) * (1.0 - p * f_e)
    n_i = p * (f_i * N) * (N - 1) * (1.0 - p * f_i)
    n_n = (1.0 - p) * N * (N - 1) * p
    return (n_e + n_i + n_n) / (N * (N - 1))
