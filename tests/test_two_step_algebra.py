"""The scalar algebra of the two-iteration PCG launch, checked on the CPU.

A two-step launch takes the second iteration's r.z and p.Ap from eleven
inner products of the basis u0 = M r, u1 = M A u0, v0 = p_prev,
v1 = M A v0 (M the Jacobi preconditioner), instead of forming the vectors
first. These expansions are identities of bilinear forms; here they are
checked against two ordinary PCG iterations (Saad, Alg. 9.1) on random SPD
systems in FP64, including a restart (beta = 0). The GPU kernel that uses
them is checked against the oracle's iterates in test_gpu_pcg."""
import numpy as np
import pytest


def sums(A, Minv, r, p):
    u0 = Minv * r
    Au0, Av0 = A @ u0, A @ p
    u1, v1 = Minv * Au0, Minv * Av0
    Au1, Av1 = A @ u1, A @ v1
    return dict(gam=r @ u0, dl=u0 @ Au0, ze=u0 @ Av0, pi=p @ Av0, a=Au0 @ u1, b=Au0 @ v1, c=Av0 @ v1,
                d=u1 @ Au1, e=Au1 @ v1, f=v1 @ Av1)


def expanded(S, gam_prev):
    """Scalars of both iterations from the sums alone (beta = 0 for a restart)."""
    beta = 0.0 if gam_prev is None else S["gam"] / gam_prev
    alpha = S["gam"] / (S["dl"] + 2 * beta * S["ze"] + beta * beta * S["pi"])
    gam1 = (S["gam"] - 2 * alpha * (S["dl"] + beta * S["ze"])
            + alpha * alpha * (S["a"] + 2 * beta * S["b"] + beta * beta * S["c"]))
    beta1 = gam1 / S["gam"]
    k = np.array([1 + beta1, -alpha, beta * beta1, -alpha * beta])
    G = np.array([[S["dl"], S["a"], S["ze"], S["b"]], [S["a"], S["d"], S["b"], S["e"]],
                  [S["ze"], S["b"], S["pi"], S["c"]], [S["b"], S["e"], S["c"], S["f"]]])
    return beta, alpha, gam1, beta1, gam1 / (k @ G @ k)


def direct(A, Minv, r, p, gam_prev):
    """Two ordinary PCG iterations from (r, p_prev)."""
    z = Minv * r
    gam = r @ z
    beta = 0.0 if gam_prev is None else gam / gam_prev
    pk = z + beta * p
    alpha = gam / (pk @ A @ pk)
    r1 = r - alpha * (A @ pk)
    z1 = Minv * r1
    gam1 = r1 @ z1
    beta1 = gam1 / gam
    pk1 = z1 + beta1 * pk
    alpha1 = gam1 / (pk1 @ A @ pk1)
    return beta, alpha, gam1, beta1, alpha1


@pytest.mark.parametrize("seed", range(6))
@pytest.mark.parametrize("restart", [False, True])
def test_expansion_matches_two_iterations(seed, restart):
    rng = np.random.default_rng(seed)
    n = 40
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.diag(rng.uniform(0.5, 3.0, n))
    Minv = 1.0 / np.diag(A)
    # a genuine CG state: run a few ordinary iterations first
    b = rng.standard_normal(n)
    r, p, gam_prev = b.copy(), np.zeros(n), None
    for _ in range(3):
        z = Minv * r
        gam = r @ z
        pk = z + (0.0 if gam_prev is None else gam / gam_prev) * p
        alpha = gam / (pk @ A @ pk)
        r, p, gam_prev = r - alpha * (A @ pk), pk, gam
    if restart:
        gam_prev = None
    got = expanded(sums(A, Minv, r, p), gam_prev)
    want = direct(A, Minv, r, p, gam_prev)
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=0)


def test_a_dropped_term_is_detected():
    """Leaving out the beta^2 c term of gamma_{k+1} changes the result far
    beyond rounding, so the check above would catch such a slip."""
    rng = np.random.default_rng(11)
    n = 30
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)
    Minv = 1.0 / np.diag(A)
    r, p = rng.standard_normal(n), rng.standard_normal(n)
    S = sums(A, Minv, r, p)
    good = expanded(S, 0.7 * S["gam"])[2]
    S_bad = dict(S, c=0.0)
    bad = expanded(S_bad, 0.7 * S["gam"])[2]
    assert abs(bad - good) > 1e-6 * abs(good)
