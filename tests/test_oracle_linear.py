"""Pin of the oracle's Kalman update + RTS smoother on a linear-Gaussian model.

The filter-smoother of Sect. 2 (gain-matrix update, RTS smoother with the
stored Jacobians) is, for a linear model, exact Gaussian conditioning.  The
reference here is the joint Gaussian of all states written out as one big
covariance matrix and conditioned on all measurements at once with numpy --
no recursion, no gain matrices, no smoother.  A dropped noise term, a
transposed Jacobian, a wrong smoother gain or a wrong chi2 changes these
numbers far beyond the tolerance.
"""
import numpy as np
import pytest

H2 = np.hstack([np.eye(2), np.zeros((2, 4))])


def _rand_spd(rng, n, scale=1.0):
    A = rng.standard_normal((n, n))
    return scale * (A @ A.T + n * np.eye(n)) / n


def _model(rng, n, with_noise=True):
    F = np.stack([np.eye(6) + 0.15 * rng.standard_normal((6, 6)) for _ in range(n)])
    Q = np.stack([_rand_spd(rng, 6, 0.05) if (with_noise and k % 3 != 1) else np.zeros((6, 6)) for k in range(n)])
    V = []
    for _ in range(n):
        Vk = _rand_spd(rng, 2, 0.2)
        V.append([Vk[0, 0], Vk[0, 1], Vk[1, 1]])
    V = np.array(V)
    x0 = 0.3 * rng.standard_normal(6)
    C0 = _rand_spd(rng, 6, 0.5)
    m = 0.3 * rng.standard_normal((n, 2))
    return F, Q, m, V, x0, C0


def _joint(F, Q, x0, C0):
    """Mean and covariance of the stacked states x_0..x_n, x_{k+1} = F_k (x_k + w_k)."""
    n = F.shape[0]
    d = 6 * (n + 1)
    mu = np.zeros(d)
    Sig = np.zeros((d, d))
    mu[:6] = x0
    Sig[:6, :6] = C0
    for k in range(n):
        a, b = slice(6 * k, 6 * k + 6), slice(6 * k + 6, 6 * k + 12)
        mu[b] = F[k] @ mu[a]
        # cross covariances with every earlier state
        Sig[b, : 6 * k + 6] = F[k] @ Sig[a, : 6 * k + 6]
        Sig[: 6 * k + 6, b] = Sig[b, : 6 * k + 6].T
        Sig[b, b] = F[k] @ (Sig[a, a] + Q[k]) @ F[k].T
    return mu, Sig


def _condition(mu, Sig, m, V, upto):
    """Condition on measurements of states 1..upto (H = [I2 0])."""
    rows = []
    for k in range(1, upto + 1):
        Hk = np.zeros((2, mu.size))
        Hk[:, 6 * k: 6 * k + 6] = H2
        rows.append(Hk)
    Hs = np.vstack(rows)
    R = np.zeros((2 * upto, 2 * upto))
    for k in range(upto):
        R[2 * k: 2 * k + 2, 2 * k: 2 * k + 2] = [[V[k, 0], V[k, 1]], [V[k, 1], V[k, 2]]]
    y = m[:upto].reshape(-1)
    Sy = Hs @ Sig @ Hs.T + R
    innov = y - Hs @ mu
    G = np.linalg.solve(Sy, Hs @ Sig).T
    post_mu = mu + G @ innov
    post_Sig = Sig - G @ Hs @ Sig
    chi2 = innov @ np.linalg.solve(Sy, innov)
    return post_mu, post_Sig, chi2


def _close(a, b, scale, tol):
    return np.max(np.abs(a - b) / scale) < tol


@pytest.mark.parametrize("seed,n,with_noise", [(1, 3, False), (2, 7, True), (3, 12, True)])
def test_linear_filter_smoother_is_gaussian_conditioning(oracle_lib, seed, n, with_noise):
    rng = np.random.default_rng(seed)
    F, Q, m, V, x0, C0 = _model(rng, n, with_noise)
    xs, Cs, xf, Cf, chi2 = oracle_lib.linear_smoother(F, Q, m, V, x0, C0)
    mu, Sig = _joint(F, Q, x0, C0)
    pm, pS, chi2_tot = _condition(mu, Sig, m, V, n)
    for k in range(n + 1):
        blk = slice(6 * k, 6 * k + 6)
        sd = np.sqrt(np.diag(pS[blk, blk]))
        assert _close(xs[k], pm[blk], sd, 1e-10), k
        assert _close(Cs[k], pS[blk, blk], np.outer(sd, sd), 1e-10), k
    # filtered state k = conditioning on measurements 1..k only
    for k in range(1, n + 1):
        fm, fS, c2k = _condition(mu, Sig, m, V, k)
        blk = slice(6 * k, 6 * k + 6)
        sd = np.sqrt(np.diag(fS[blk, blk]))
        assert _close(xf[k - 1], fm[blk], sd, 1e-10), k
        assert _close(Cf[k - 1], fS[blk, blk], np.outer(sd, sd), 1e-10), k
        # prediction-error decomposition: sum of chi2 increments = innovation form
        assert abs(chi2[:k].sum() - c2k) < 1e-10 * max(1.0, c2k)
    assert abs(chi2.sum() - chi2_tot) < 1e-10 * max(1.0, chi2_tot)


def test_smoother_gain_is_inverse_jacobian_without_noise(oracle_lib):
    """Q = 0: x_{k|n} = F_k^{-1} x_{k+1|n} (the RTS gain reduces to F^{-1})."""
    rng = np.random.default_rng(7)
    F, Q, m, V, x0, C0 = _model(rng, 6, with_noise=False)
    xs, Cs, xf, Cf, chi2 = oracle_lib.linear_smoother(F, Q, m, V, x0, C0)
    for k in range(6):
        back = np.linalg.solve(F[k], xs[k + 1])
        sd = np.sqrt(np.diag(Cs[k]))
        assert _close(xs[k], back, sd, 1e-9)
        Cb = np.linalg.solve(F[k], np.linalg.solve(F[k], Cs[k + 1]).T)
        assert _close(Cs[k], Cb, np.outer(sd, sd), 1e-9)


def _condition_rows(mu, Sig, rows, R, y):
    """Condition N(mu, Sig) on y = Hs x + e, e ~ N(0, R) (Hs = stacked rows)."""
    Hs = np.vstack(rows)
    Sy = Hs @ Sig @ Hs.T + R
    G = np.linalg.solve(Sy, Hs @ Sig).T
    return mu + G @ (y - Hs @ mu), Sig - G @ Hs @ Sig


@pytest.mark.parametrize("seed,n,with_noise,scale", [(4, 3, False, 1e3), (5, 8, True, 1e2), (6, 12, True, 1e4)])
def test_linear_two_filter_is_conditioning_with_a_weak_prior(oracle_lib, seed, n, with_noise, scale):
    """Two-filter smoother (Sect. 2, Fig. 2) on a linear-Gaussian model.

    Its backward filter starts from the last filtered state x_{n|n} with
    covariance scale * C_{n|n}.  With a backward model x_k = G_k x_{k+1} - w_k
    (G_k = F_k^{-1}) the backward transition density equals the forward one,
    so the combined estimate of state k < n is the joint Gaussian conditioned
    on every measurement plus one extra observation y = x_{n|n} of state n with
    covariance scale * C_{n|n}; state n itself is the filtered state.  Because
    y equals the posterior mean of state n, the extra observation moves no
    mean: the means are the RTS means, and only the covariances shrink, by a
    part of order 1/scale."""
    rng = np.random.default_rng(seed)
    F, Q, m, V, x0, C0 = _model(rng, n, with_noise)
    # component 2 is the azimuth, which the update and the combination wrap
    # into (-pi, pi]: scale the means down so that the weakly constrained
    # backward predictions stay far inside that range (the model is linear,
    # so this changes nothing else)
    m, x0 = 0.05 * m, 0.05 * x0
    G = np.linalg.inv(F)
    xs2, Cs2 = oracle_lib.linear_two_filter(F, G, Q, m, V, x0, C0, scale)
    xs, Cs, _, _, _ = oracle_lib.linear_smoother(F, Q, m, V, x0, C0)
    mu, Sig = _joint(F, Q, x0, C0)
    pm, pS, _ = _condition(mu, Sig, m, V, n)
    last = slice(6 * n, 6 * n + 6)
    rows, R = [], np.zeros((2 * n + 6, 2 * n + 6))
    for k in range(1, n + 1):
        Hk = np.zeros((2, mu.size))
        Hk[:, 6 * k: 6 * k + 6] = H2
        rows.append(Hk)
        R[2 * k - 2: 2 * k, 2 * k - 2: 2 * k] = [[V[k - 1, 0], V[k - 1, 1]], [V[k - 1, 1], V[k - 1, 2]]]
    Hy = np.zeros((6, mu.size))
    Hy[:, last] = np.eye(6)
    rows.append(Hy)
    R[2 * n:, 2 * n:] = scale * pS[last, last]
    y = np.concatenate([m.reshape(-1), pm[last]])
    am, aS = _condition_rows(mu, Sig, rows, R, y)
    for k in range(n + 1):
        blk = slice(6 * k, 6 * k + 6)
        ref_m, ref_S = (pm[blk], pS[blk, blk]) if k == n else (am[blk], aS[blk, blk])
        sd = np.sqrt(np.diag(ref_S))
        assert _close(xs2[k], ref_m, sd, 1e-9), k
        assert _close(Cs2[k], ref_S, np.outer(sd, sd), 1e-9), k
        assert _close(xs2[k], xs[k], sd, 1e-9), k
    # the covariance difference to RTS is the weak prior's share, of order 1/scale
    d = max(np.max(np.abs(Cs2[k] - Cs[k]) / np.outer(np.sqrt(np.diag(Cs[k])), np.sqrt(np.diag(Cs[k]))))
            for k in range(n))
    assert 1e-3 / scale < d < 10.0 / scale
