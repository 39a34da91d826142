"""Seeded synthetic inputs, shared by the tests, the benchmark and the smoke check.

Holds no step of the factorisation or the solve: only the construction of the SPD test
matrices and right-hand sides.  Every generator is numpy PCG64 (default_rng) from an
explicit seed, so the oracle and the device path see identical bits.

Workloads (all synthetic; the paper names no dataset for its Cholesky runs):
  * lower_plus_shift   A = L0 L0^T + n I, L0 = tril(U[-1,1]) (diagonal included), b ~ U[-1,1]
  * gram_spd           A = G G^T / n + I, G ~ N(0,1); eigenvalues in about [1, 5]
  * known_factor       A = L0 L0^T with L0_ii = n + U[0,1], off-diagonal U[-1,1]
  * integer_factor     A = L0 L0^T with small-integer L0 and diagonal in {1,2,4} (or unit
                       diagonal and entries in {-1,0,1}): every intermediate of an
                       in-place Cholesky is then an exact integer
  * haar_spd           A = Q diag(s) Q^T, Q Haar (QR of a Gaussian matrix with the signs
                       of diag(R) folded in), s log-uniform on [1, kappa] with both
                       endpoints pinned, symmetrised
  * reflector_spd      as haar_spd but Q a product of k Householder reflectors (exactly
                       orthogonal; a cheap stand-in for Haar at large sizes)
  * batch_sizes        sizes and right-hand-side counts of the batched workload
  * request_stream     the arrival process and request shapes of the serving workload
"""
import math

import numpy as np


def rng(seed):
    return np.random.default_rng(seed)


def lower_plus_shift(n, seed=1):
    g = rng(seed)
    L0 = np.tril(g.uniform(-1.0, 1.0, (n, n)))
    A = L0 @ L0.T + n * np.eye(n)
    b = g.uniform(-1.0, 1.0, n)
    return A, b


def gram_spd(n, seed=2, nrhs=1):
    g = rng(seed)
    G = g.standard_normal((n, n))
    A = G @ G.T / n + np.eye(n)
    B = g.standard_normal((n, nrhs))
    return A, B


def gram_factor_G(n, seed=2, nrhs=1):
    """The raw draws of gram_spd (G and the right-hand sides), for callers that form
    G G^T / n + I on the device: same stream, so the same A up to the product's rounding."""
    g = rng(seed)
    G = g.standard_normal((n, n))
    B = g.standard_normal((n, nrhs))
    return G, B


def known_factor(n, seed=3):
    g = rng(seed)
    L0 = np.tril(g.uniform(-1.0, 1.0, (n, n)), -1)
    L0[np.diag_indices(n)] = n + g.uniform(0.0, 1.0, n)
    return L0 @ L0.T, L0


def integer_factor(n, seed=4, nrhs=2, unit=False):
    """unit=True: unit diagonal and off-diagonal entries in {-1, 0, 1} (a quarter each
    sign); then the inverse of every 32x32 diagonal block is also an integer matrix
    (entries below 2^31), so block-inverse based solves stay exact too."""
    g = rng(seed)
    if unit:
        L0 = np.tril(g.choice([-1.0, 0.0, 0.0, 1.0], (n, n)), -1)
        L0[np.diag_indices(n)] = 1.0
        X0 = g.integers(-5, 6, (n, nrhs)).astype(np.float64)
        A = L0 @ L0.T
        return A, L0, X0, A @ X0
    L0 = np.tril(g.integers(-3, 4, (n, n)).astype(np.float64), -1)
    L0[np.diag_indices(n)] = g.choice([1.0, 2.0, 4.0], n)
    X0 = g.integers(-5, 6, (n, nrhs)).astype(np.float64)
    A = L0 @ L0.T
    return A, L0, X0, A @ X0


def log_spectrum(n, kappa, g):
    s = np.exp(g.uniform(0.0, math.log(kappa), n))
    if n >= 2:
        s[0], s[-1] = 1.0, float(kappa)
    return s


def haar_q(n, g):
    Z = g.standard_normal((n, n))
    Q, R = np.linalg.qr(Z)
    return Q * np.sign(np.diag(R))


def haar_spd(n, kappa, seed=5, nrhs=1):
    g = rng(seed)
    Q = haar_q(n, g)
    s = log_spectrum(n, kappa, g)
    A = (Q * s) @ Q.T
    A = (A + A.T) / 2
    B = g.standard_normal((n, nrhs))
    return A, B


def reflectors(n, k, g):
    V = g.standard_normal((n, k))
    return V / np.linalg.norm(V, axis=0)


def apply_reflectors_sym(D, V):
    """Q diag(D) Q^T for Q = H_1 ... H_k, H_i = I - 2 v_i v_i^T."""
    n = len(D)
    A = np.diag(D).astype(np.float64)
    for i in range(V.shape[1] - 1, -1, -1):
        v = V[:, i]
        Av = A @ v
        A = A - 2.0 * np.outer(v, Av) - 2.0 * np.outer(Av, v) + 4.0 * (v @ Av) * np.outer(v, v)
    A = (A + A.T) / 2
    assert A.shape == (n, n)
    return A


def reflector_spd(n, kappa, seed=6, nrhs=1, k=8):
    g = rng(seed)
    V = reflectors(n, k, g)
    s = log_spectrum(n, kappa, g)
    A = apply_reflectors_sym(s, V)
    B = g.standard_normal((n, nrhs))
    return A, B


def batch_sizes(count=4096, lo=32, hi=512, rhs_lo=1, rhs_hi=8, seed=7):
    g = rng(seed)
    n = g.integers(lo, hi + 1, count)
    q = g.integers(rhs_lo, rhs_hi + 1, count)
    return n.astype(np.int64), q.astype(np.int64)


def batch_matrix(n, seed, nrhs):
    """Member of the batched workload: A = G G^T / n + I, right-hand sides N(0,1)."""
    return gram_spd(int(n), seed=int(seed), nrhs=int(nrhs))


def request_stream(count=20000, rate=2000.0, n_lo=64, n_hi=8192, rhs_lo=1, rhs_hi=64,
                   kappa_lo=1e1, kappa_hi=1e6, seed=8):
    """Poisson arrivals; n log-uniform, nrhs uniform, condition number log-uniform."""
    g = rng(seed)
    t = np.cumsum(g.exponential(1.0 / rate, count))
    n = np.round(np.exp(g.uniform(math.log(n_lo), math.log(n_hi), count))).astype(np.int64)
    q = g.integers(rhs_lo, rhs_hi + 1, count).astype(np.int64)
    kappa = np.exp(g.uniform(math.log(kappa_lo), math.log(kappa_hi), count))
    seeds = g.integers(0, 2**31 - 1, count).astype(np.int64)
    return {"t": t, "n": n, "nrhs": q, "kappa": kappa, "seed": seeds}
