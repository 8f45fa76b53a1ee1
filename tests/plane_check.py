"""Parity check of plane-regularised covariances (Segal et al., cited in the
sparsity-aware paragraph of Sec. III-A.2): Sigma = I + (eps - 1) n n^T with n
a unit vector of the smallest eigenspace of the neighbourhood's sample
covariance.  Shared by the GPU parity test and its CPU pin."""
import numpy as np

EPS = 1e-3


def mats(c6):
    c = np.asarray(c6, dtype=np.float64)
    return np.stack([np.stack([c[0], c[1], c[2]], -1), np.stack([c[1], c[3], c[4]], -1),
                     np.stack([c[2], c[4], c[5]], -1)], -2)


def assert_plane_parity(g6, o6, eq1_6, valid, what, say=print):
    """g6: covariances under test, o6: the oracle's, eq1_6: the oracle's Eq. (1)
    covariances of the same neighbourhoods (a positive multiple of the sample
    covariance plus 1e-3 I, so the same eigenvectors and proportional gaps).

    Where the smallest eigenvalue is separated from the next by more than
    1e-4 of the largest, the normal is unique and g6 must equal o6 to float
    rounding.  Elsewhere every unit vector of the smallest eigenspace is a
    correct normal: n, the eigenvector of g6's eps eigenvalue, must satisfy
    n^T E n - lambda_min(E) <= (lambda_mid - lambda_min) + 2e-6 lambda_max,
    which a normal outside that eigenspace fails unless lambda_max is within
    2e-6 of lambda_mid (then every unit vector is correct).  Every valid
    point also has the spectrum {eps, 1, 1}; invalid points are zero."""
    G, O, E = mats(g6), mats(o6), mats(eq1_6)
    v = valid != 0
    assert np.all(G[~v] == 0)
    lam = np.linalg.eigvalsh(E[v])
    unique = (lam[:, 1] - lam[:, 0]) > 1e-4 * lam[:, 2]
    d = np.abs(G[v] - O[v]).max(axis=(1, 2))
    if unique.any():
        assert np.all(d[unique] <= 2e-6), (what, float(d[unique].max()))
    spec = np.linalg.eigvalsh(G[v])
    np.testing.assert_allclose(spec, np.broadcast_to([EPS, 1.0, 1.0], spec.shape), rtol=0,
                               atol=2e-6)
    nu = ~unique
    excess = np.zeros(0)
    if nu.any():
        _, Q = np.linalg.eigh(G[v][nu])
        n = Q[:, :, 0]
        q = np.einsum("pi,pij,pj->p", n, E[v][nu], n)
        lu = lam[nu]
        excess = (q - lu[:, 0]) - ((lu[:, 1] - lu[:, 0]) + 2e-6 * lu[:, 2])
        assert np.all(excess <= 0), (what, "normal outside the smallest eigenspace",
                                     int((excess > 0).sum()), float(excess.max()))
    say(f"{what}: {int(v.sum())} valid, {int(unique.sum())} with a unique normal, "
        f"{int(nu.sum())} checked on the smallest eigenspace, max diff "
        f"{float(d[unique].max()) if unique.any() else 0.0:.2e}")
    return int(unique.sum()), int(nu.sum())
