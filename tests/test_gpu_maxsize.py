"""A grid past 32-bit byte offsets: 2560x1920x110 (540,672,000 unknowns), where every FP64 grid
array is 4.3 GB.  The tridiagonal kernel takes its generic path (64-bit level offsets) there;
the SpMV, the tridiagonal solve and a short FP64 solve are checked against the oracle on
sampled rows / columns and by the oracle's full FP64 product."""
import numpy as np
import pytest

import synth
from tests.helpers import host

pytestmark = pytest.mark.gpu

EPS64 = 2.0 ** -53


def test_arrays_beyond_4gib(oracle_mod):
    import torch
    import paper_1811_03852_amd as eg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    eg.load_library()
    torch.cuda.empty_cache()
    # 110 levels with the top/bottom layer-thickness ratio of the 70-level recipe
    p = synth.Problem(2560, 1920, 110, ratio=1.1 ** (69.0 / 109.0), seed=5, name="maxsize_2560x1920x110")
    assert p.n * 8 > 2 ** 32
    coef = synth.make_coeffs(p, threads=16)
    print(f"[maxsize] {p.nlon}x{p.nlat}x{p.nlev} generated", flush=True)
    op = eg.Operator(torch.from_numpy(coef).cuda())
    torch.cuda.synchronize()
    try:
        rng = np.random.default_rng(41)
        x = rng.standard_normal(p.n)
        corners = [i + p.nlon * (j + p.nlat * k) for i in (0, p.nlon - 1) for j in (0, p.nlat - 1)
                   for k in (0, p.nlev // 2, p.nlev - 1)]
        idx = np.unique(np.concatenate([rng.integers(0, p.n, 5000), corners, [p.n - 1]]))
        ref = oracle_mod.apply_points(coef, x, idx)
        y = host(op.apply(torch.from_numpy(x).cuda()))[idx]
        scale = 2.0 * coef[6].reshape(-1)[idx] * np.max(np.abs(x))
        print(f"[maxsize] SpMV max |y - oracle| / scale = {np.max(np.abs(y - ref) / scale):.2e}", flush=True)
        assert np.all(np.abs(y - ref) <= 32 * EPS64 * scale)

        # tridiagonal solve on sampled columns (the last column reaches the end of every array)
        P = p.nlon * p.nlat
        cols = np.unique(np.concatenate([rng.integers(0, P, 1000), [0, p.nlon - 1, P - p.nlon, P - 1]]))
        z = host(op.precond(torch.from_numpy(x).cuda())).reshape(p.nlev, P)[:, cols].ravel()
        nlat, nlon = coef.shape[2:]
        sub = np.ascontiguousarray(coef[:, :, cols // nlon, cols % nlon][:, :, None, :])
        qin = x.reshape(p.nlev, P)[:, cols].ravel()
        zref = oracle_mod.thomas(sub, qin)
        rel = np.max(np.abs(z - zref)) / np.max(np.abs(zref))
        print(f"[maxsize] Thomas max rel diff to oracle {rel:.2e}", flush=True)
        assert rel <= 1e-10

        # a short FP64 solve: the library's true residual against the oracle's full product
        b = synth.make_rhs(p).ravel()
        xs = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(torch.from_numpy(b).cuda(), xs, 1e-3, 2000, eg.FP64)
        true_rel = np.linalg.norm(b - oracle_mod.apply(coef, host(xs))) / np.linalg.norm(b)
        print(f"[maxsize] FP64 to 1e-3: status {info.status}, {info.iterations} its, {info.seconds:.2f} s, "
              f"true R (oracle) {true_rel:.3e}, library {info.true_rel_residual:.3e}", flush=True)
        assert info.status == eg.CONVERGED and true_rel <= 1e-3
        assert abs(true_rel - info.true_rel_residual) <= 1e-6 * true_rel
    finally:
        op.close()
        torch.cuda.empty_cache()
