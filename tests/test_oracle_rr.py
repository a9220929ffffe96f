"""Pin of the recursive-regularized model's higher-order terms (orders three
and up), independent of the oracle's pair-sum loop.

The model assembles f_out_k = t_k sum_{n in S} H_n(c_k) A_n / N_n over the
weighted Hermite polynomials H_n (per axis 1, c, c^2 - 1/3) of its support set
S. Projecting the output, p_m = sum_k H_m(c_k) f_out_k = sum_n G_mn A_n / N_n
with the Gram matrix G_mn = sum_k t_k H_m H_n (diagonal on D3Q27; on D3Q19 the
third-order members overlap), recovers the coefficients A_n. For |n| >= 2
they must be
    rho u^n + 1/2 sum_ab Pi*_ab d^2(u^n)/(du_a du_b),
the second-derivative form of the pair-sum recursion (each pair of the n
indices contributes Pi* times the product of u over the other indices), with
Pi* the relaxed non-equilibrium stress (Eq. bulk)."""
import itertools

import numpy as np
import pytest

from paper_2010_11751_amd import workloads as W


def support(q):
    out = []
    for n in itertools.product(range(3), repeat=3):
        order = sum(n)
        if q == 27 or order <= 2 or (order == 3 and sorted(n) == [0, 1, 2]):
            out.append(n)
    return out


def hermite(n, c):
    h = np.ones(len(c))
    for a in range(3):
        x = c[:, a].astype(float)
        h = h * (1.0 if n[a] == 0 else x if n[a] == 1 else x * x - 1.0 / 3.0)
    return h


def monomial_second_derivative(n, a, b, u):
    """d^2(prod_g u_g^{n_g}) / (du_a du_b) at u."""
    e = list(n)
    coef = 1.0
    for d in (a, b):
        if e[d] == 0:
            return 0.0
        coef *= e[d]
        e[d] -= 1
    return coef * float(np.prod([u[g] ** e[g] for g in range(3)]))


@pytest.mark.parametrize("q", (19, 27))
@pytest.mark.parametrize("omega,omega_bulk", [(1.4, None), (1.85, 1.1)])
def test_rr_hermite_coefficients_follow_the_recursion(orc, q, omega, omega_bulk):
    c, t, _ = orc.lattice(q)
    cfg = orc.Config(q=q, model=orc.RR, omega=omega, omega_bulk=omega_bulk)
    wb = omega if omega_bulk is None else omega_bulk
    S = support(q)
    G = np.array([[float((t * hermite(m, c) * hermite(n, c)).sum()) for n in S] for m in S])
    norm = np.array([np.prod([(1.0, 1.0 / 3.0, 2.0 / 9.0)[k] for k in n]) for n in S])
    if q == 27:   # the full tensor basis is orthogonal, with the Hermite norms
        assert np.abs(G - np.diag(norm)).max() < 1e-15
    for f in W.random_populations(23, q, 4):
        rho = f.sum()
        u = (c.T.astype(float) @ f) / rho
        Pi = np.einsum("k,ka,kb->ab", f, c.astype(float), c.astype(float)) - rho * np.outer(u, u) - rho * np.eye(3) / 3
        tr = np.trace(Pi) / 3
        Ps = (1 - omega) * (Pi - tr * np.eye(3)) + (1 - wb) * tr * np.eye(3)
        fo = orc.collide(cfg, f)
        proj = np.array([float(hermite(m, c) @ fo) for m in S])
        A = norm * np.linalg.solve(G, proj)
        for j, n in enumerate(S):
            if sum(n) < 2:
                continue
            got = A[j]
            un = rho * float(np.prod([u[g] ** n[g] for g in range(3)]))
            want = un + 0.5 * sum(Ps[a, b] * monomial_second_derivative(n, a, b, u)
                                  for a in range(3) for b in range(3))
            assert abs(got - want) < 2e-15, n
