"""Graph replay of the batched BiCGStab iterations (option graph) against kernel-by-kernel
launches: the same solution and residual history bit for bit, replay after replay with other
work on the stream in between, in every plain mode and with both preconditioners; a change of
option between solves takes a graph of its own; and the launch-overhead gain on a small grid."""
import time

import numpy as np
import pytest

import synth
from tests.helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eg():
    import torch
    import paper_1811_03852_amd as eg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    eg.load_library()
    return eg


@pytest.fixture(scope="module")
def small():
    p = synth.CONFIGS["small_96x72x20"]
    return p, synth.make_coeffs(p), synth.make_rhs(p).ravel()


def _solve(eg, op, p, b, mode, tol):
    import torch
    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
    info = op.solve(b, x, tol, 20000, mode)
    return host(x), op.history(), info


CASES = [("FP64", 0), ("FP64", 1), ("FP32_IR", 0), ("FP32_IR", 1), ("FP32_IR_BF16", 1), ("FP32_IR_FP16", 0),
         ("FP32_MP", 0), ("FP32_MP", 1)]


@pytest.mark.parametrize("mode_name,precond", CASES, ids=[f"{m}-{'sor' if c else 'tri'}" for m, c in CASES])
def test_graph_replays_match_launches(eg, oracle_mod, small, mode_name, precond):
    import torch
    p, coef, bh = small
    tol = 1e-6 if mode_name == "FP32_MP" else 1e-8
    mode = getattr(eg, mode_name)
    b = dev(bh)
    with eg.Operator(dev(coef)) as op:
        op.set_option("precond", precond)
        runs = []
        for graph in (0, 1, 1, 0, 1):
            op.set_option("graph", graph)
            runs.append(_solve(eg, op, p, b, mode, tol))
            y = op.apply(b)               # other work on the operator's stream between solves
            assert torch.isfinite(y).all()
    x0, h0, i0 = runs[0]
    assert i0.status == eg.CONVERGED
    rel = np.linalg.norm(bh - oracle_mod.apply(coef, x0)) / np.linalg.norm(bh)
    assert rel <= tol
    for x, h, info in runs[1:]:
        assert (info.status, info.iterations, info.outer_steps, info.restarts) == \
               (i0.status, i0.iterations, i0.outer_steps, i0.restarts)
        assert np.array_equal(x, x0) and np.array_equal(h, h0)


def test_option_change_takes_its_own_graph(eg, small):
    """Line-SOR sweeps 3, then 2, with graphs: each solve equals the launched solve with the
    same option (a stale graph would keep the three sweeps)."""
    p, coef, bh = small
    b = dev(bh)
    out = {}
    with eg.Operator(dev(coef)) as op:
        op.set_option("precond", 1)
        for graph in (1, 0):
            op.set_option("graph", graph)
            for sweeps in (3, 2):
                op.set_option("sor_sweeps", sweeps)
                out[graph, sweeps] = _solve(eg, op, p, b, eg.FP64, 1e-8)
    for sweeps in (3, 2):
        assert np.array_equal(out[1, sweeps][0], out[0, sweeps][0])
        assert out[1, sweeps][2].iterations == out[0, sweeps][2].iterations
    assert not np.array_equal(out[1, 3][0], out[1, 2][0])


def test_graph_cuts_launch_overhead_on_a_small_grid(eg, small):
    """96x72x20 in FP64 (launch-bound): the median of five solves with and without graphs."""
    import torch
    p, coef, bh = small
    b = dev(bh)
    with eg.Operator(dev(coef)) as op:
        times = {}
        for graph in (0, 1):
            op.set_option("graph", graph)
            _solve(eg, op, p, b, eg.FP64, 1e-8)
            ts = []
            for _ in range(5):
                x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                info = op.solve(b, x, 1e-8, 20000, eg.FP64)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
            times[graph] = (sorted(ts)[2], info.iterations)
    print(f"96x72x20 FP64: launches {times[0][0] * 1e3:.2f} ms, graph {times[1][0] * 1e3:.2f} ms "
          f"({times[1][1]} iterations, {times[1][0] / times[1][1] * 1e6:.1f} us per iteration)")
    assert times[0][1] == times[1][1]


def test_graph_option_is_checked(eg, small):
    p, coef, _ = small
    with eg.Operator(dev(coef)) as op:
        for bad in (2, 0.5, -1):
            with pytest.raises(eg.EndgameError):
                op.set_option("graph", bad)
        op.set_option("graph", 0)
        op.set_option("graph", 1)
