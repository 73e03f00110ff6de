"""FP64 noise floor of a parity comparison, measured with the oracle alone.

Two FP64 implementations that sum in different orders differ by rounding.
Galerkin entries are sums of 5^d * 3^d products with heavy cancellation (rows
sum to zero), so their rounding error is of the order of one ulp of the row's
largest entry times sqrt(number of terms), not one ulp of the entry itself; at
coefficient contrast 1e4 the BoxMG step from level 2 to level 1 amplifies that
to 1e-11..1e-10 in the weights.  The oracle is therefore run once as is and
once with such noise injected into every Galerkin product (and, separately,
with one-ulp noise on every intermediate vector of the cycle); a GPU/oracle
comparison passes when it is within SAFETY times the larger of the two
distances, and never needs to be tighter than the stated floor."""
import numpy as np
import scipy.linalg as sla

import oracle as O

SAFETY = 20.0


def _row_noise(seed, d):
    rng = np.random.default_rng(seed)
    amp = 2.0 ** -52 * np.sqrt(float(3 ** d * 5 ** d))

    def f(Ac):
        Ac = Ac.tocsr(copy=True)
        rm = np.asarray(abs(Ac).max(axis=1).todense()).ravel()
        rows = np.repeat(np.arange(Ac.shape[0]), np.diff(Ac.indptr))
        Ac.data = Ac.data + amp * rm[rows] * rng.uniform(-1.0, 1.0, size=Ac.data.shape)
        return Ac
    return f


def perturbed_hierarchies(p, transfer, seeds=(101, 102), check_definite=True):
    return [O.build_hierarchy(p.eps, p.dim, p.level, transfer=transfer, perturb=_row_noise(s, p.dim),
                              check_definite=check_definite)
            for s in seeds]


def _noisy_vcycle(H, l, u, b, rng):
    def ulp(x):
        return x * (1.0 + 2.0 ** -52 * rng.uniform(-1.0, 1.0, size=x.shape))
    A = H.A[l]
    D = A.diagonal()
    if l == H.lc:
        return ulp(sla.lu_solve(H.coarse_lu, b))
    for _ in range(H.mu_pre):
        u = ulp(O.jacobi(A, D, u, b, H.omega))
    r = ulp(b - A @ u)
    P = H.P[l]
    ec = _noisy_vcycle(H, l - 1, np.zeros(P.shape[1]), ulp(P.T @ r), rng)
    u = ulp(u + P @ ec)
    for _ in range(H.mu_post):
        u = ulp(O.jacobi(A, D, u, b, H.omega))
    return u


def iterate_tolerances(p, transfer, H, cycles, floor=1e-12):
    """Bounds for ||A (u_gpu - u_oracle)|| / ||b|| after each of ``cycles``
    cycles (an array, cycle 1 first), and the oracle's last iterate.  By the
    triangle inequality they also bound the difference of the two relative
    residuals of that cycle."""
    b = O.rhs_from_f(p.f, p.dim, p.level)
    A = H.A[p.level]
    nb = np.linalg.norm(b)

    def iterates(step):
        u, out = np.zeros_like(b), []
        for _ in range(cycles):
            u = step(u)
            out.append(u)
        return out

    base = iterates(lambda u: O.vcycle(H, p.level, u, b))
    worst = np.zeros(cycles)
    runs = []
    if transfer != "geometric":
        runs = [lambda u, Hp=Hp: O.vcycle(Hp, p.level, u, b) for Hp in perturbed_hierarchies(p, transfer)]
        if H.coarse_lu is not None:
            rng = np.random.default_rng(7)
            runs.append(lambda u: _noisy_vcycle(H, p.level, u, b, rng))
    for step in runs:
        for j, up in enumerate(iterates(step)):
            worst[j] = max(worst[j], np.linalg.norm(A @ (base[j] - up)) / nb)
    return np.maximum(floor, SAFETY * worst), base[-1]


def operator_tolerance(p, transfer, H, floor=1e-12, check_definite=True):
    """Per level: absolute bound for P weights, relative bound for stencils."""
    tolP, tolA = {}, {}
    for Hp in perturbed_hierarchies(p, transfer, check_definite=check_definite):
        for l in H.P:
            dP = abs(H.P[l] - Hp.P[l]).max() if l in Hp.P else 0.0
            tolP[l] = max(tolP.get(l, floor), SAFETY * dP)
        for l in H.A:
            if l in Hp.A:
                dA = abs(H.A[l] - Hp.A[l]).max() / abs(H.A[l]).max()
                tolA[l] = max(tolA.get(l, floor), SAFETY * dA)
    return tolP, tolA
