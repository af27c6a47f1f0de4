"""Weighted CP-ALS on the GPU (thc_cp_als; Sec. II.c-d Eq. 15-16, 21, Appendix I Eq. 43-46)
against the oracle's exact-solve ALS from the same start: the factors after each run of sweeps and
the objective after every sweep.  The GPU solves each update's normal equations by conjugate
gradients preconditioned with diag(S) to a relative residual of 1e-13, so the factors agree to the
solve's accuracy times the conditioning of S (random factors: well conditioned)."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_11473_amd import thc
    thc.load()
    return thc


def _case(seed, I, J, K, n, planted, weights, noise=1e-2):
    rng = np.random.default_rng(seed)
    if planted:
        A = np.einsum("in,jn,kn->ijk", rng.standard_normal((I, planted)), rng.standard_normal((J, planted)),
                      rng.standard_normal((K, planted)))
        A += noise * rng.standard_normal((I, J, K))
    else:
        A = rng.standard_normal((I, J, K))
    X, Y, Z = (rng.standard_normal((m, n)) for m in (I, J, K))
    w = [None, None, None]
    for d, m in enumerate((I, J, K)):
        if weights[d] == "rand":
            w[d] = rng.uniform(0.2, 1.5, m)
        elif weights[d] == "decay":  # eigenvalue-like weights (Eq. 15): a few large, a long small tail
            w[d] = np.sqrt(np.exp(-np.arange(m) / (0.2 * m)))
        elif weights[d] == "zero":  # a weight of zero: that slice does not enter the other updates
            w[d] = rng.uniform(0.5, 1.0, m)
            w[d][m // 2] = 0.0
    return A, X, Y, Z, w


CASES = [
    # seed, I, J, K, n, planted rank, weights of the three indices, sweeps
    (1, 5, 7, 11, 3, 3, ("rand", "rand", "rand"), 4),
    (2, 13, 11, 37, 9, 0, (None, None, None), 3),
    (3, 9, 9, 150, 20, 6, (None, None, "decay"), 3),  # Eq. 15 shape: ia pairs x rank, eigenvalue weights on P
    (4, 17, 17, 200, 70, 0, ("rand", "rand", None), 2),  # Eq. 21 shape: occupation weights on the orbitals
    (5, 150, 33, 140, 131, 0, ("zero", "rand", "zero"), 2),  # n above two GEMM tiles, ragged
]


@pytest.mark.parametrize("case", CASES, ids=[f"s{c[0]}_{c[1]}x{c[2]}x{c[3]}_n{c[4]}" for c in CASES])
def test_cp_als_matches_the_oracle(lib, case):
    import torch
    from oracle import cpals
    seed, I, J, K, n, planted, weights, sweeps = case
    print(f"[gpu-cpals] {case}", flush=True)
    A, X, Y, Z, w = _case(seed, I, J, K, n, planted, weights)
    Xo, Yo, Zo, obj_o = cpals.cp_als(A, X, Y, Z, sweeps, *w)
    dev = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device="cuda").contiguous()
    Ad, Xd, Yd, Zd = dev(A), dev(X), dev(Y), dev(Z)
    obj, its = lib.cp_als(Ad, Xd, Yd, Zd, sweeps, *(dev(x) for x in w), cg_tol=1e-13, cg_maxit=2000)
    torch.cuda.synchronize()
    print(f"[gpu-cpals] most CG iterations {its}; objective gpu {obj} oracle {obj_o}", flush=True)
    for name, got, ref in (("X", Xd, Xo), ("Y", Yd, Yo), ("Z", Zd, Zo)):
        g = got.cpu().numpy()
        err = np.abs(g - ref).max() / np.abs(ref).max()
        assert err < 1e-8, (name, err)
    scale = obj_o[0]
    for a, b in zip(obj, obj_o):
        assert abs(a - b) <= 1e-10 * scale + 1e-9 * abs(b), (a, b)
    assert all(obj[k + 1] <= obj[k] * (1 + 1e-12) + 1e-14 * scale for k in range(sweeps))


def test_cp_als_zero_sweeps_and_no_objective(lib):
    """Zero sweeps leave the factors as given and report the start's objective; without the
    objective array the factors after a sweep are still those of the oracle."""
    import torch
    from oracle import cpals
    A, X, Y, Z, w = _case(7, 6, 5, 8, 4, 0, ("rand", None, "rand"))
    dev = lambda a: None if a is None else torch.tensor(a, dtype=torch.float64, device="cuda").contiguous()
    Ad, Xd, Yd, Zd = dev(A), dev(X), dev(Y), dev(Z)
    obj, its = lib.cp_als(Ad, Xd, Yd, Zd, 0, *(dev(x) for x in w))
    assert its == 0 and len(obj) == 1
    assert abs(obj[0] - cpals.objective(A, X, Y, Z, *w)) <= 1e-12 * obj[0]
    assert np.array_equal(Xd.cpu().numpy(), X) and np.array_equal(Zd.cpu().numpy(), Z)
    obj, _ = lib.cp_als(Ad, Xd, Yd, Zd, 1, *(dev(x) for x in w), cg_tol=1e-13, objective=False)
    assert obj is None
    Xo, Yo, Zo, _ = cpals.cp_als(A, X, Y, Z, 1, *w)
    for got, ref in ((Xd, Xo), (Yd, Yo), (Zd, Zo)):
        assert np.abs(got.cpu().numpy() - ref).max() < 1e-8 * np.abs(ref).max()


def test_cp_als_rejects_bad_arguments(lib):
    import torch
    A = torch.zeros((2, 2, 2), dtype=torch.float64, device="cuda")
    F = torch.zeros((2, 1), dtype=torch.float64, device="cuda")
    with pytest.raises(lib.ThcError):
        lib.cp_als(A, F, F, F, 1, cg_tol=0.0)
    with pytest.raises(lib.ThcError):
        lib.cp_als(A, F, F, F, -1)
