"""Learned preconditioner on the GPU: network parity with the FP64 oracle (forward and
gradients), harvests, training, flexible BiCGStab and FGMRES, the stall fallback and the
trained network's gain."""
import numpy as np
import pytest

import synth
from oracle import net as onet
from tests.helpers import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def eg():
    import torch
    import paper_1811_03852_amd as eg
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    eg.load_library()
    return eg


def _theta(seed, w4_scale=0.3):
    rng = np.random.default_rng(seed)
    d = onet.unpack(onet.init_theta(seed))
    d["W4"] = rng.standard_normal(d["W4"].shape) * w4_scale
    d["b1"] = rng.standard_normal(32) * 0.1
    d["b2"] = rng.standard_normal(32) * 0.1
    d["b3"] = rng.standard_normal(32) * 0.1
    d["b4"] = np.array([0.02])
    # the GPU keeps FP32 master weights: the oracle sees the same FP32 values
    return onet.pack(d).astype(np.float32).astype(np.float64)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


# 32x6x9 and 48x7x20 take the layered inference with the 3x3 kernel for rows of whole
# 16-position tiles (nlon % 16 == 0); 64x6x9, 128x5x12 and 192x9x70 (nlon % 64 == 0) the
# one-launch inference, whose last block of four rows is partly outside the grid
@pytest.mark.parametrize("p", [synth.Problem(24, 12, 9, seed=2), synth.Problem(37, 9, 20, seed=3),
                               synth.Problem(32, 6, 9, seed=4), synth.Problem(48, 7, 20, seed=5),
                               synth.Problem(64, 6, 9, seed=6), synth.Problem(128, 5, 12, seed=7),
                               synth.Problem(192, 9, 70, seed=8)],
                         ids=lambda p: f"{p.nlon}x{p.nlat}x{p.nlev}")
def test_forward_matches_oracle(eg, p):
    import torch
    coef = synth.make_coeffs(p)
    th = _theta(4)
    net = eg.Net(0)
    net.set_weights(th.astype(np.float32))
    q = np.random.default_rng(5).standard_normal(p.n).astype(np.float32)
    with eg.Operator(dev(coef)) as op:
        delta = torch.empty(p.n, dtype=torch.float32, device="cuda")
        z = host(net.apply(op, dev(q), delta)).astype(np.float64)
    d_ref, _ = onet.forward(th, coef, q.astype(np.float64), bf16_round=True)
    z_ref = onet.apply(th, coef, q.astype(np.float64), bf16_round=True)
    dg = host(delta).astype(np.float64)
    e_d, e_z = _rel(dg, d_ref), _rel(z, z_ref)
    # per level, against the level-average size of delta: an error confined to a few levels
    # (a column chunk's boundary levels, say) shows here even when the total is small
    per_level = np.linalg.norm((dg - d_ref).reshape(p.nlev, -1), axis=1) / (np.linalg.norm(d_ref) / np.sqrt(p.nlev))
    print(f"forward parity: delta rel L2 {e_d:.2e} (worst level {per_level.max():.2e}), M(q) rel L2 {e_z:.2e}")
    assert e_d <= 1e-3 and per_level.max() <= 2e-3 and e_z <= 5e-4
    net.close()


# nlon a multiple of 64: 64x6x9 and 192x9x70 leave the last four-row block partly outside the
# grid, 128x1x3 has one row (both neighbours are poles) and fewer levels than taps, 256x8x20
# spans several blocks in both directions
@pytest.mark.parametrize("shape", [(64, 6, 9), (128, 1, 3), (192, 9, 70), (256, 8, 20)],
                         ids=lambda s: "x".join(map(str, s)))
def test_fused_inference_is_the_layered_one_bitwise(eg, shape):
    """The one-launch inference (option net_fused 1) against the layer-by-layer kernels
    (net_fused 0): the same delta and M(q) bit for bit, and learned solves in FP64 and in FP32
    with refinement that follow the same trajectory bit for bit."""
    import torch
    p = synth.Problem(*shape, seed=11)
    coef = synth.make_coeffs(p)
    net = eg.Net(0)
    net.set_weights(_theta(5).astype(np.float32))
    q = dev(np.random.default_rng(6).standard_normal(p.n).astype(np.float32))
    b = dev(synth.make_rhs(p).ravel())
    with eg.Operator(dev(coef)) as op:
        out = {}
        for fused in (1, 0):
            op.set_option("net_fused", fused)
            delta = torch.empty(p.n, dtype=torch.float32, device="cuda")
            z = net.apply(op, q, delta)
            op.attach(net)
            op.set_option("learned_method", 0)
            sols = []
            for mode in (eg.LEARNED_FP64, eg.LEARNED_FP32_IR):
                x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
                info = op.solve(b, x, 1e-10, 12, mode)
                sols.append((x, op.history(), info.iterations))
            op.attach(None)
            out[fused] = (z, delta, sols)
        z1, d1, s1 = out[1]
        z0, d0, s0 = out[0]
        assert torch.equal(d1, d0) and torch.equal(z1, z0)
        assert float(torch.linalg.vector_norm(d1)) > 0.0
        for (x1, h1, i1), (x0, h0, i0) in zip(s1, s0):
            assert i1 == i0 and torch.equal(x1, x0) and np.array_equal(h1, h0)
    net.close()


# the second shape gives every gradient workgroup two or three chunks of 32 positions (the
# chunk pipeline's both halves and its early exit), a ragged last chunk and a ragged last batch
# of levels in the column kernels
@pytest.mark.parametrize("shape", [(24, 12, 9), (47, 31, 30)], ids=lambda s: "x".join(map(str, s)))
@pytest.mark.parametrize("kind", [onet.LOSS_ERROR, onet.LOSS_RESIDUAL])
def test_gradients_match_oracle(eg, kind, shape):
    p = synth.Problem(*shape, seed=6)
    coef = synth.make_coeffs(p)
    th = _theta(7)
    net = eg.Net(0)
    net.set_weights(th.astype(np.float32))
    net.set_loss(kind)
    rng = np.random.default_rng(8)
    r = rng.standard_normal(p.n).astype(np.float32)
    e = rng.standard_normal(p.n).astype(np.float32)
    with eg.Operator(dev(coef)) as op:
        L, g = net.loss_grad(op, dev(r), dev(e))
    L_ref, g_ref = onet.loss_and_grad(th, coef, r.astype(np.float64), e.astype(np.float64), bf16_round=True,
                                      kind=kind)
    assert abs(L - L_ref) <= 1e-3 * abs(L_ref)
    G, Gr = onet.unpack(g.astype(np.float64)), onet.unpack(g_ref)
    worst = 0.0
    for name, _ in onet.SHAPES:
        err = _rel(G[name].ravel(), Gr[name].ravel())
        print(f"grad {name}: rel L2 {err:.2e}")
        worst = max(worst, err)
    assert worst <= 5e-3
    net.close()


@pytest.mark.parametrize("kind", [onet.LOSS_ERROR, onet.LOSS_RESIDUAL])
def test_training_steps_match_oracle_adam(eg, kind):
    """eg_net_train from known weights: two pairs in one batch of two, two epochs, so two Adam
    steps on the mean gradient of the pairs.  The oracle takes the same two steps with its FP64
    gradient (loss_and_grad) and its Adam (adam_step, Kingma & Ba's Algorithm 1); the updates
    theta_2 - theta_0 agree element by element wherever the gradient is well above the BF16
    gradient error, and are bounded by the Adam step size everywhere else."""
    import torch
    p = synth.Problem(24, 12, 9, seed=6)
    coef = synth.make_coeffs(p)
    th0 = _theta(7)
    rng = np.random.default_rng(12)
    r = rng.standard_normal((2, p.n)).astype(np.float32)
    e = rng.standard_normal((2, p.n)).astype(np.float32)
    lr = 1e-2
    net = eg.Net(0)
    net.set_weights(th0.astype(np.float32))
    net.set_loss(kind)
    with eg.Operator(dev(coef)) as op:
        net.train([op], dev(r), dev(e), [0, 0], epochs=2, batch=2, lr=lr, seed=0)
        th2_gpu = net.get_weights().astype(np.float64)
    net.close()
    st = onet.AdamState(th0.size)
    th, grads = th0, []
    for _ in range(2):
        gs = [onet.loss_and_grad(th, coef, r[i].astype(np.float64), e[i].astype(np.float64), bf16_round=True,
                                 kind=kind)[1] for i in range(2)]
        g = 0.5 * (gs[0] + gs[1])
        grads.append(g)
        th = onet.adam_step(th, g, st, lr)
    u_ref, u_gpu = th - th0, th2_gpu - th0
    # a parameter is well determined when both of its gradients stand 25x above the noise of the
    # BF16 gradient (relative L2 error per tensor about 2e-4, so 2e-4 of the tensor's rms)
    ok = np.ones(th0.size, dtype=bool)
    o = 0
    for _, shape in onet.SHAPES:
        size = int(np.prod(shape))
        for g in grads:
            seg = g[o:o + size]
            ok[o:o + size] &= np.abs(seg) > 5e-3 * np.sqrt(np.mean(seg * seg))
        o += size
    dev_ok = np.max(np.abs(u_gpu[ok] - u_ref[ok]))
    rel_ok = np.linalg.norm(u_gpu[ok] - u_ref[ok]) / np.linalg.norm(u_ref[ok])
    print(f"Adam steps: {ok.mean():.1%} of parameters well determined, there max |du| {dev_ok / lr:.2e} lr, "
          f"rel L2 {rel_ok:.2e}; max |u| {np.max(np.abs(u_gpu)) / lr:.3f} lr")
    assert ok.mean() >= 0.65
    # a wrong bias correction, swapped decay rates or a wrong batch mean move these by O(lr)
    assert dev_ok <= 5e-2 * lr and rel_ok <= 1e-2, (dev_ok, rel_ok)
    # two Adam steps move no parameter by more than about 2 lr
    assert np.max(np.abs(u_gpu)) <= 2.05 * lr


def test_flexible_bicgstab_follows_oracle(eg, oracle_mod):
    """EG_LEARNED_FP64 with flexible BiCGStab (learned_method 0) against the oracle's flexible
    BiCGStab (oracle/krylov.bicgstab_flex) driven by the oracle's network (oracle/net.apply,
    BF16 rounding where the GPU stores BF16) with the same stall fallback to T^{-1}.  This random
    network makes both stall and fall back once, after the same number of iterations; the first
    iteration's two residuals agree to the network's rounding, the iteration counts agree
    closely, x agrees to the tolerance's conditioning, and the GPU's recursive residual is its
    true one (x advanced along exactly the preconditioned vectors that entered A).
    Later history entries are not compared one by one: with a nonlinear M the recurrence loses
    its bi-orthogonality and the trajectory is chaotic (the oracle's own third residual moves by
    11 % when M's output is perturbed by 1e-5 relative)."""
    import torch
    from oracle import krylov
    p = synth.Problem(48, 24, 10, seed=7)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    th = _theta(4, 0.3)
    x_or, ref = krylov.bicgstab_flex(coef, b, lambda q: onet.apply(th, coef, q, bf16_round=True), tol=1e-10,
                                     fallback=lambda q: oracle_mod.thomas(coef, q), stall_window=20)
    assert ref.status == 0
    net = eg.Net(0)
    net.set_weights(th.astype(np.float32))
    with eg.Operator(dev(coef)) as op:
        op.attach(net)
        op.set_option("learned_method", 0)
        op.set_option("stall_window", 20)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-10, 5000, eg.LEARNED_FP64)
        h = op.history()
    net.close()
    xh = host(x)
    k = 2
    dh = np.abs(h[:k] - ref.history[:k]) / ref.history[:k]
    err = np.linalg.norm(xh - x_or) / np.linalg.norm(x_or)
    print(f"flexible BiCGStab: GPU {info.iterations} its {info.fallbacks} fallbacks, oracle {ref.iterations} its "
          f"{ref.fallbacks} fallbacks; first {k} history entries agree to {dh.max():.2e}; x error {err:.2e}")
    assert info.status == eg.CONVERGED and info.fallbacks == ref.fallbacks
    assert abs(info.iterations - ref.iterations) <= max(3, ref.iterations // 10)
    assert dh.max() <= 1e-4
    assert err <= 1e-8
    assert abs(info.true_rel_residual - h[-1]) <= 1e-12


def test_learned_pc_train_save_load(eg, oracle_mod):
    """The operator-owned learned preconditioner through the C ABI: learned modes refuse to run
    before it exists (EG_ENOPC); eg_train_learned_pc harvests pairs from the operator's own FP64
    solves and lowers the error-space loss on pairs it did not train on; the saved image loads
    into a second operator bit for bit, and both solve to the same x bit for bit; a damaged
    image is refused."""
    import torch
    p = synth.Problem(48, 24, 10, seed=9)
    coef = synth.make_coeffs(p)
    b = dev(synth.make_rhs(p, seed=77).ravel())
    with eg.Operator(dev(coef)) as op:
        x1 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        with pytest.raises(eg.EndgameError) as exc:
            op.solve(b, x1, 1e-8, 2000, eg.LEARNED_FP64)
        assert exc.value.code == eg.ENOPC
        with pytest.raises(eg.EndgameError):
            op.save_learned_pc()
        r, e = op.harvest(b, 12)                  # held-out pairs (another right-hand side)
        owner = [0] * r.shape[0]
        base = eg.Net(0)                          # zero output layer: M = T^{-1}
        base.set_loss(eg.Net.LOSS_ERROR)
        loss0 = base.eval([op], r, e, owner)
        base.close()
        op.train_learned_pc("source=iterates,rhs=4,pairs=12,loss=error,batch=8", epochs=15, lr=2e-3, seed=3)
        loss1 = op.learned_pc().eval([op], r, e, owner)
        print(f"eg_train_learned_pc: held-out error-space loss {loss0:.4f} (T^-1 alone) -> {loss1:.4f}")
        assert loss1 < loss0
        img = op.save_learned_pc()
        assert len(img) == eg.PC_IMAGE_BYTES and img[:4] == b"EGPC"
        i1 = op.solve(b, x1, 1e-8, 2000, eg.LEARNED_FP64)
        rel = np.linalg.norm(host(b) - oracle_mod.apply(coef, host(x1))) / np.linalg.norm(host(b))
        assert i1.status == eg.CONVERGED and rel <= 1e-8
    with eg.Operator(dev(coef)) as op2:
        op2.load_learned_pc(img)
        assert op2.save_learned_pc() == img
        x2 = torch.zeros_like(x1)
        i2 = op2.solve(b, x2, 1e-8, 2000, eg.LEARNED_FP64)
        assert i2.iterations == i1.iterations and torch.equal(x1, x2)
        bad = bytearray(img)
        bad[4] = 2                                # format version 2 does not exist
        with pytest.raises(eg.EndgameError) as exc:
            op2.load_learned_pc(bytes(bad))
        assert exc.value.code == eg.EINVAL
        with pytest.raises(eg.EndgameError):
            op2.load_learned_pc(img[:-4])
        with pytest.raises(eg.EndgameError):
            op2.train_learned_pc("source=nowhere")


def test_zero_output_layer_reproduces_plain_solver_bitwise(eg):
    """Untrained net (zero output layer): delta = 0 exactly, so flexible BiCGStab with the
    learned M follows the tridiagonal-preconditioned trajectory bit for bit."""
    import torch
    p = synth.CONFIGS["small_96x72x20"]
    coef = synth.make_coeffs(p)
    b = dev(synth.make_rhs(p).ravel())
    net = eg.Net(3)
    with eg.Operator(dev(coef)) as op:
        op.attach(net)
        op.set_option("learned_method", 0)
        for plain, learned in ((eg.FP64, eg.LEARNED_FP64), (eg.FP32_IR, eg.LEARNED_FP32_IR)):
            x1 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
            i1 = op.solve(b, x1, 1e-8, 5000, plain)
            h1 = op.history()
            x2 = torch.zeros_like(x1)
            i2 = op.solve(b, x2, 1e-8, 5000, learned)
            h2 = op.history()
            assert i1.status == i2.status == eg.CONVERGED
            assert torch.equal(x1, x2) and np.array_equal(h1, h2) and i2.fallbacks == 0
    net.close()


def test_zero_output_layer_fgmres_is_plain_fgmres_bitwise(eg):
    """Same identity for FGMRES: with delta = 0 the learned modes run plain FGMRES."""
    import torch
    p = synth.CONFIGS["small_96x72x20"]
    coef = synth.make_coeffs(p)
    b = dev(synth.make_rhs(p).ravel())
    net = eg.Net(3)
    with eg.Operator(dev(coef)) as op:
        op.attach(net)
        op.set_option("method", 1)
        op.set_option("learned_method", 1)
        for plain, learned in ((eg.FP64, eg.LEARNED_FP64), (eg.FP32_IR, eg.LEARNED_FP32_IR)):
            x1 = torch.zeros(p.n, dtype=torch.float64, device="cuda")
            i1 = op.solve(b, x1, 1e-8, 5000, plain)
            h1 = op.history()
            x2 = torch.zeros_like(x1)
            i2 = op.solve(b, x2, 1e-8, 5000, learned)
            h2 = op.history()
            assert i1.status == i2.status == eg.CONVERGED
            assert torch.equal(x1, x2) and np.array_equal(h1, h2) and i2.fallbacks == 0
    net.close()


def test_harvest_pairs(eg, oracle_mod):
    p = synth.Problem(48, 24, 10, seed=9)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    with eg.Operator(dev(coef)) as op:
        r, e = op.harvest(dev(b), 12)
    assert r.shape[0] == 12
    rh, eh = host(r).astype(np.float64), host(e).astype(np.float64)
    assert np.array_equal(rh[0], b.astype(np.float32).astype(np.float64))   # snapshot 0: x0 = 0
    for i in (0, 5, 11):
        # r_i = b - A x_i and e_i = x* - x_i with A x* = b  =>  r_i = A e_i (up to FP32 rounding)
        Ae = oracle_mod.apply(coef, eh[i])
        assert _rel(Ae, rh[i]) <= 1e-4
    # the iterates converge: errors shrink
    assert np.linalg.norm(eh[11]) < 0.1 * np.linalg.norm(eh[0])


def test_harvest_krylov_pairs(eg, oracle_mod):
    """The Krylov harvest stores an orthonormal basis starting at b / ||b|| and A^{-1} of each."""
    import torch
    p = synth.Problem(48, 24, 10, seed=9)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    with eg.Operator(dev(coef)) as op:
        r, e = op.harvest_krylov(dev(b), 12)
        r2, none = op.harvest_krylov(dev(b), 5, errors=False)
    assert r.shape[0] == 12 and none is None
    rh, eh = host(r).astype(np.float64), host(e).astype(np.float64)
    assert np.allclose(rh[0], b / np.linalg.norm(b), rtol=0, atol=1e-6)
    G = rh @ rh.T
    assert np.max(np.abs(G - np.eye(12))) <= 1e-5          # orthonormal to FP32 rounding
    assert torch.equal(r2, r[:5])                              # the basis does not depend on nvec
    for i in (0, 6, 11):
        # e is stored in FP32: A e reproduces v to about cond(A) x 6e-8 (shift 1e-3: cond ~ 1e3)
        assert _rel(oracle_mod.apply(coef, eh[i]), rh[i]) <= 1e-4


@pytest.fixture(scope="module")
def trained(eg):
    """A network trained (residual-space loss) on the Krylov bases of eight small operators of
    the generator's family."""
    import torch
    ops, rs, es, owner = [], [], [], []
    for s in range(8):
        p = synth.Problem(48, 24, 10, seed=1000 + s)
        op = eg.Operator(dev(synth.make_coeffs(p)))
        b = synth.make_rhs(p, seed=2000 + s).ravel()
        r, e = op.harvest_krylov(dev(b), 20)
        ops.append(op)
        rs.append(r)
        es.append(e)
        owner += [s] * r.shape[0]
    r = torch.cat(rs).contiguous()
    e = torch.cat(es).contiguous()
    net = eg.Net(11)
    loss0 = net.eval(ops, r, e, owner)
    hist = net.train(ops, r, e, owner, epochs=20, batch=16, lr=2e-3, seed=1)
    yield dict(net=net, ops=ops, r=r, e=e, owner=owner, loss0=loss0, hist=hist)
    for op in ops:
        op.close()
    net.close()


def test_training_reduces_loss(trained):
    h = trained["hist"]
    print(f"loss untrained {trained['loss0']:.4f}, per epoch {np.round(h, 4)}")
    assert trained["loss0"] == pytest.approx(h[0], rel=0.5)
    assert h[-1] < 0.5 * trained["loss0"]


def test_training_is_deterministic(eg, trained):
    ops, r, e, owner = trained["ops"], trained["r"], trained["e"], trained["owner"]
    w = []
    for _ in range(2):
        net = eg.Net(11)
        net.train(ops, r, e, owner, epochs=2, batch=8, lr=2e-3, seed=1)
        w.append(net.get_weights())
        net.close()
    assert np.array_equal(w[0], w[1])


@pytest.mark.parametrize("method", [0, 1], ids=["bicgstab", "fgmres"])
@pytest.mark.parametrize("mode_name", ["LEARNED_FP64", "LEARNED_FP32_IR"])
def test_learned_modes_reach_1e8(eg, oracle_mod, trained, mode_name, method):
    import torch
    p = synth.Problem(48, 24, 10, seed=1017)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p, seed=2017).ravel()
    x_ref, _ = oracle_mod.bicgstab(coef, b, tol=1e-12)
    with eg.Operator(dev(coef)) as op:
        op.attach(trained["net"])
        op.set_option("learned_method", method)
        x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
        info = op.solve(dev(b), x, 1e-8, 5000, getattr(eg, mode_name))
        xp = torch.zeros_like(x)
        plain = op.solve(dev(b), xp, 1e-8, 5000, eg.FP64)
    xh = host(x)
    rel = np.linalg.norm(b - oracle_mod.apply(coef, xh)) / np.linalg.norm(b)
    err = np.linalg.norm(xh - x_ref) / np.linalg.norm(x_ref)
    print(f"{mode_name} method {method}: iterations {info.iterations} (plain FP64 {plain.iterations}), "
          f"fallbacks {info.fallbacks}, "
          f"true R {rel:.2e}, error vs oracle {err:.2e}")
    assert info.status == eg.CONVERGED and rel <= 1e-8 and err <= 1e-5


def test_trained_network_gain(eg, oracle_mod, trained):
    """What the trained network gains over the method without it, on operators it never saw:
    FGMRES(30) with M = T^{-1}(q + rho delta(q)) against FGMRES(30) with T^{-1} (asserted: at
    least 10 % fewer iterations), and the time-to-solve of every combination against BiCGStab
    with T^{-1}, the solver the network is meant to beat (reported: on these grids the network's
    cost per application outweighs the iterations it saves)."""
    import time
    import torch
    rows = []
    for k in range(3):
        p = synth.Problem(48, 24, 10, seed=7777 + k)
        coef = synth.make_coeffs(p)
        b = synth.make_rhs(p, seed=8888 + k).ravel()
        x_or, info_or = oracle_mod.bicgstab(coef, b, tol=1e-8)
        with eg.Operator(dev(coef)) as op:
            op.attach(trained["net"])
            row = {"oracle_bicgstab": info_or.iterations}
            for method, name in ((1, "fgmres"), (0, "bicgstab")):
                op.set_option("method", method)
                op.set_option("learned_method", method)
                for mode, tag in ((eg.FP64, "tri"), (eg.LEARNED_FP64, "learned")):
                    x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
                    op.solve(dev(b), x, 1e-8, 5000, mode)          # untimed: buffers
                    x.zero_()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    info = op.solve(dev(b), x, 1e-8, 5000, mode)
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    rel = np.linalg.norm(b - oracle_mod.apply(coef, host(x))) / np.linalg.norm(b)
                    assert info.status == eg.CONVERGED and rel <= 1e-8
                    row[f"{name}_{tag}"] = (info.iterations, info.fallbacks, dt)
            rows.append(row)
            print(f"held-out operator {k}: " + ", ".join(f"{key} {val}" for key, val in row.items()))
    tri = np.mean([r["fgmres_tri"][0] for r in rows])
    learned = np.mean([r["fgmres_learned"][0] for r in rows])
    print(f"FGMRES iterations: T^-1 {tri:.1f}, learned {learned:.1f} ({100 * (1 - learned / tri):.0f}% fewer)")
    base = np.mean([r["bicgstab_tri"][2] for r in rows])
    for key in ("fgmres_tri", "fgmres_learned", "bicgstab_learned"):
        print(f"time-to-solve {key}: {np.mean([r[key][2] for r in rows]) / base:.2f} x BiCGStab with T^-1 "
              f"({1e3 * base:.2f} ms)")
    assert learned <= 0.9 * tri and all(r["fgmres_learned"][1] == 0 for r in rows)


def test_stall_triggers_fallback_and_still_converges(eg, oracle_mod):
    """A network with large random output weights is a poor preconditioner: the stall rule
    switches to T^{-1} and the solve still reaches the tolerance."""
    import torch
    p = synth.Problem(48, 24, 10, seed=21)
    coef = synth.make_coeffs(p)
    b = synth.make_rhs(p).ravel()
    net = eg.Net(0)
    net.set_weights(_theta(13, w4_scale=30.0).astype(np.float32))
    with eg.Operator(dev(coef)) as op:
        op.attach(net)
        op.set_option("stall_window", 5)
        for mode in (eg.LEARNED_FP64, eg.LEARNED_FP32_IR):
            x = torch.zeros(p.n, dtype=torch.float64, device="cuda")
            info = op.solve(dev(b), x, 1e-8, 5000, mode)
            rel = np.linalg.norm(b - oracle_mod.apply(coef, host(x))) / np.linalg.norm(b)
            assert info.fallbacks >= 1 and info.status == eg.CONVERGED and rel <= 1e-8, info
    net.close()
