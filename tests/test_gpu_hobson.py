"""The Hobson / spherical-tensor route to the Hermite integrals
(f12_hermite_hobson; Sec. II.D, Eq. (Ylm) with the Laplacian powers of
Eq. (QxQyQz) restored) against the oracle's MD recurrence on the same
radial derivatives.  Both are exact expressions of d^t_x d^u_y d^v_z B in
A_j = D^j B at X, and A_j can take any values (a radial B with those
derivatives exists), so they must agree for random A_j.  Without the
(nabla^2)^k factors every R_tuv with t + u + v >= 2 would differ."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1412_5070_amd import f12int
    return f12int


@pytest.mark.parametrize("L", [0, 2, 4, 8, 12, 14])
def test_hobson_route_equals_md_recurrence(lib, L):
    import torch
    from oracle import dd
    from oracle.hermite import hermite_r
    rng = np.random.default_rng(100 + L)
    npt = 24
    A = rng.uniform(-1.0, 1.0, (npt, L + 1))
    X = rng.uniform(-1.5, 1.5, (npt, 3))
    X[0] = 0.0  # Q = P: only even t, u, v survive
    R = lib.hermite_hobson(torch.as_tensor(A, device="cuda"), torch.as_tensor(X, device="cuda"), L).cpu().numpy()
    cube = hermite_r(dd.DD(A), dd.DD(X[:, 0]), dd.DD(X[:, 1]), dd.DD(X[:, 2]), L).to_float()
    worst = 0.0
    h = 0
    for N in range(L + 1):
        idx = []
        for t in range(N, -1, -1):
            for u in range(N - t, -1, -1):
                idx.append((h, t, u, N - t - u))
                h += 1
        got = np.stack([R[:, i] for (i, _, _, _) in idx], 1)
        want = np.stack([cube[:, t, u, v] for (_, t, u, v) in idx], 1)
        # scale of order N: the largest |R| of that order at the point (and 1e-300 for an all-zero order)
        sc = np.maximum(np.max(np.abs(want), axis=1), 1e-300)
        err = np.max(np.abs(got - want), axis=1) / sc
        worst = max(worst, float(err.max()))
        assert np.all(err < 1e-11), (N, float(err.max()))
    print(f"Hobson vs MD, L={L}: worst error relative to the order's largest |R| {worst:.2e}", flush=True)
