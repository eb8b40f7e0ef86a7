"""Learned-start network on the GPU vs its FP64 oracle (bf16 rounding emulated at the same points)."""
import numpy as np
import pytest
import torch

from oracle import cnn_oracle as C
from oracle import recon_oracle as O
from synth import generators as G

pytestmark = pytest.mark.gpu


def dev():
    return torch.device("cuda", 0)


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev())


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / np.linalg.norm(b))


def sample(n, seed, box=200.0, observer=(37.0, -60.0, 110.0)):
    rng = np.random.default_rng(seed)
    delta = O.smooth(rng.standard_normal((n, n, n)), box, 2.0 * box / n).astype(np.float32)
    u_p = (O.smooth(rng.standard_normal((n, n, n)), box, 2.0 * box / n) * 40).astype(np.float32)
    target = (-0.15 * u_p + rng.standard_normal((n, n, n)) * 0.2).astype(np.float32)
    rhat = O.line_of_sight(n, box, (0, 0, 0), observer)
    return delta, u_p, target, rhat


def params(seed):
    th = C.init_params(seed)
    th[-1] = 0.05
    return th.astype(np.float32)


@pytest.mark.parametrize("n", [16, 32])
def test_forward_matches_oracle(gpu_lib, n):
    from paper_1504_02591_amd import native
    box, obs = 200.0, (37.0, -60.0, 110.0)
    delta, u_p, _, rhat = sample(n, 10 + n, box, obs)
    th = params(3)
    plan = native.Plan(n, box, obs, 2.0, 0.7, 0.0, randoms=False, cnn=True)
    du = plan.cnn_forward(to_dev(th), to_dev(delta), to_dev(u_p))[0].cpu().numpy()
    plan.close()
    y, _ = C.forward(th.astype(np.float64), delta.astype(np.float64), u_p.astype(np.float64), rhat, bf16_mode=True)
    e = rel_l2(du, y / C.S_U)
    print(f"n={n} forward rel L2 {e:.2e}", flush=True)
    assert e < 1e-3


def test_loss_and_gradient_match_oracle(gpu_lib):
    from paper_1504_02591_amd import native
    n, box, obs = 16, 200.0, (37.0, -60.0, 110.0)
    delta, u_p, target, rhat = sample(n, 5, box, obs)
    th = params(4)
    plan = native.Plan(n, box, obs, 2.0, 0.7, 0.0, randoms=False, cnn=True)
    grad = torch.zeros(native.CNN_PARAMS, dtype=torch.float32, device=dev())
    loss = plan.cnn_train_step(to_dev(th), None, None, 0, 0.0, to_dev(delta), to_dev(u_p), to_dev(target),
                               grad_out=grad)
    plan.close()
    ref_loss, ref_grad = C.loss_and_grad(th.astype(np.float64), delta.astype(np.float64), u_p.astype(np.float64),
                                         rhat, target.astype(np.float64), bf16_mode=True)
    g = grad.cpu().numpy()
    print(f"loss gpu {loss:.6e} oracle {ref_loss:.6e}", flush=True)
    assert abs(loss - ref_loss) <= 1e-4 * ref_loss
    off = 0
    for name, shp in C.SHAPES:
        size = int(np.prod(shp))
        e = rel_l2(g[off:off + size], ref_grad[off:off + size])
        print(f"grad {name}: rel L2 {e:.2e}", flush=True)
        assert e < 5e-3, name
        off += size


def test_adam_update_gpu(gpu_lib):
    from paper_1504_02591_amd import native
    n, box, obs = 16, 200.0, (37.0, -60.0, 110.0)
    delta, u_p, target, rhat = sample(n, 6, box, obs)
    th0 = params(5)
    th = to_dev(th0)
    m = torch.zeros_like(th)
    v = torch.zeros_like(th)
    grad = torch.zeros_like(th)
    plan = native.Plan(n, box, obs, 2.0, 0.7, 0.0, randoms=False, cnn=True)
    for step in (1, 2):
        before = th.cpu().numpy().astype(np.float64)
        mb, vb = m.cpu().numpy().astype(np.float64), v.cpu().numpy().astype(np.float64)
        plan.cnn_train_step(th, m, v, step, 1e-3, to_dev(delta), to_dev(u_p), to_dev(target), grad_out=grad)
        exp, _, _ = C.adam_step(before, mb, vb, grad.cpu().numpy().astype(np.float64), step, 1e-3)
        np.testing.assert_allclose(th.cpu().numpy(), exp, rtol=1e-5, atol=1e-7)
    plan.close()


def test_training_reduces_loss(gpu_lib):
    from paper_1504_02591_amd import native
    n, box, obs = 32, 300.0, (150.0, 150.0, 150.0)
    delta, u_p, target, _ = sample(n, 7, box, obs)
    th = to_dev(params(6))
    m, v = torch.zeros_like(th), torch.zeros_like(th)
    plan = native.Plan(n, box, obs, 2.0, 0.7, 0.0, randoms=False, cnn=True)
    d, u, t = to_dev(delta), to_dev(u_p), to_dev(target)
    first = plan.cnn_train_step(th, m, v, 1, 3e-3, d, u, t)
    for step in range(2, 201):
        last = plan.cnn_train_step(th, m, v, step, 3e-3, d, u, t)
    plan.close()
    print(f"loss {first:.4e} -> {last:.4e}", flush=True)
    assert last < 0.3 * first


def ffta2_weights(growth, bias):
    """Weights whose output is exactly the FFTA-2 correction -c u_p (relu(x) - relu(-x) = x)."""
    beta = growth / bias
    c = 3 * beta / (7 + 3 * beta)
    p = C.unpack(np.zeros(C.N_PARAMS))
    p["W1"][0, 13, 1] = 1.0
    p["W1"][1, 13, 1] = -1.0
    p["W2"][0, 13, 0] = 1.0
    p["W2"][1, 13, 1] = 1.0
    p["W3"][0, 13, 0] = -c
    p["W3"][0, 13, 1] = c
    return C.pack(p)


def test_learned_start_end_to_end(gpu_lib):
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 21, 22, ran_factor=3, bias=1.2, smooth_r=20.0)
    th = params(8)
    th[:] = 0.5 * th + 0.5 * ffta2_weights(cat.growth, cat.bias).astype(np.float32)
    for npass in (1, 3):
        plan = native.plan_for(cat, keep_delta=True, start_buffers=True, cnn=True)
        gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
        plan.paint(native.GAL, gal)
        plan.paint(native.RAN, ran)
        plan.solve(native.START_LEARNED, to_dev(th))
        rc, iters, eps = plan.iterate(npass, 0.0)
        psi = plan.psi()[0].cpu().numpy()
        plan.close()
        grid_g = O.paint(cat.gal_pos, None, cat.n, cat.box_len, cat.origin)
        grid_r = O.paint(cat.ran_pos, None, cat.n, cat.box_len, cat.origin)
        delta = O.overdensity(grid_g, grid_r, cat.box_len, cat.smooth_r, cat.mask_tau)
        rhat = O.line_of_sight(cat.n, cat.box_len, cat.origin, cat.observer)
        plain = O.reconstruct_field(delta, cat.box_len, cat.origin, cat.observer, cat.bias, cat.growth, n_passes=0)
        u_p = np.sum(plain["psi"] * rhat, axis=0)
        y, _ = C.forward(th.astype(np.float64), C.bf16(delta), u_p, rhat, bf16_mode=True)
        ref = O.reconstruct_field(delta, cat.box_len, cat.origin, cat.observer, cat.bias, cat.growth,
                                  n_passes=npass, start=O.START_LEARNED, start_correction=y / C.S_U)
        e = rel_l2(psi, ref["psi"])
        print(f"learned start {npass} passes: psi rel L2 {e:.2e}, eps {eps[0]} vs {ref['eps']}", flush=True)
        assert e < 1e-4
        np.testing.assert_allclose(eps[0], ref["eps"], rtol=1e-3, atol=1e-5)


def test_learned_start_split_calls_equal_one_call(gpu_lib):
    # solve leaves the combined fan-out of the start; iterate(0) rebuilds state X from D_s for the
    # output, and the next call starts the learned pass from there: same passes bit for bit.  A call
    # that ends right after the start pass resolves eps_1 from the output's fan-out instead of the
    # next pass's z step: the same sum rounded along another path.
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.7, 23, 24, ran_factor=3, bias=1.2, smooth_r=20.0)
    th = params(9)
    th[:] = 0.5 * th + 0.5 * ffta2_weights(cat.growth, cat.bias).astype(np.float32)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    out = []
    for split in ((3,), (0, 2, 1), (0, 1, 2)):
        plan = native.plan_for(cat, keep_delta=True, start_buffers=True, cnn=True)
        plan.paint(native.GAL, gal)
        plan.paint(native.RAN, ran)
        plan.solve(native.START_LEARNED, to_dev(th))
        eps, psis = [], []
        for k in split:
            rc, iters, e = plan.iterate(k, 0.0)
            eps += list(e[0])
            psis.append(plan.psi()[0].cpu().numpy())
        out.append((iters[0], eps, psis))
        plan.close()
    (i1, e1, p1), (i2, e2, p2), (i3, e3, p3) = out
    assert i1 == i2 == i3 == 3
    assert e1 == e2 and e1[1:] == e3[1:]
    assert abs(e3[0] - e1[0]) <= 1e-6 * e1[0]
    assert np.array_equal(p1[-1], p2[-1]) and np.array_equal(p1[-1], p3[-1])
    # iterate(0) after the learned solve returns the plain start's displacement
    plain = native.plan_for(cat, keep_delta=True)
    plain.paint(native.GAL, gal)
    plain.paint(native.RAN, ran)
    plain.solve()
    plain.iterate(0, 0.0)
    p0 = plain.psi()[0].cpu().numpy()
    plain.close()
    assert np.array_equal(p2[0], p0)


@pytest.mark.parametrize("n", [32, 128])
def test_restrict_and_prolong_match_oracle(gpu_lib, n):
    from paper_1504_02591_amd import native
    b = 2
    rng = np.random.default_rng(11)
    f = rng.standard_normal((b, n, n, n)).astype(np.float32)
    c = rng.standard_normal((b, n // 2, n // 2, n // 2)).astype(np.float32)
    plan = native.Plan(n, 100.0, (0.0, 0.0, 0.0), 1.0, 0.5, 0.0, batch=b, randoms=False)
    rc = plan.restrict(to_dev(f)).cpu().numpy()
    pc = plan.prolong(to_dev(c)).cpu().numpy()
    plan.close()
    for i in range(b):
        np.testing.assert_allclose(rc[i], C.restrict(f[i]), rtol=0, atol=2e-6)
        np.testing.assert_allclose(pc[i], C.prolong(c[i]), rtol=0, atol=1e-6)


@pytest.mark.parametrize("n,levels", [(32, 1), (64, 1), (64, 2), (128, 2), (256, 2)])
def test_learned_start_coarse_grid_end_to_end(gpu_lib, n, levels):
    # network on the (n/2)^3 (RECON_CNN_HALF) or (n/4)^3 (RECON_CNN_QUARTER) grid: inputs restricted,
    # output prolonged (level by level below the quarter grid's one-pass trilinear prolongation)
    from paper_1504_02591_amd import native
    # at 256^3 the survey geometry (beta = 0.37), with a network closer to the FFTA-2 map so that the
    # plain start does not provably beat it and it is kept
    th = params(9)
    if n >= 256:
        cat = G.config2(n=n, scale=n / 512.0, seeds=(71, 72, 73))
        th[:] = 0.2 * th + 0.8 * ffta2_weights(cat.growth, cat.bias).astype(np.float32)
    else:
        cat = G.lattice_box(n, 500.0, (-500.0, 250.0, 250.0), 0.7, 23, 24, ran_factor=3, bias=1.2, smooth_r=20.0)
        th[:] = 0.5 * th + 0.5 * ffta2_weights(cat.growth, cat.bias).astype(np.float32)
    plan = native.plan_for(cat, keep_delta=True, start_buffers=True, cnn=True, cnn_half=levels == 1,
                           cnn_quarter=levels == 2)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve(native.START_LEARNED, to_dev(th))
    rc, iters, eps = plan.iterate(2, 0.0)
    psi = plan.psi()[0].cpu().numpy()
    assert plan.restarts() == [0]
    plan.close()
    grid_g = O.paint(cat.gal_pos, None, cat.n, cat.box_len, cat.origin)
    grid_r = O.paint(cat.ran_pos, None, cat.n, cat.box_len, cat.origin)
    delta = O.overdensity(grid_g, grid_r, cat.box_len, cat.smooth_r, cat.mask_tau)
    rhat = O.line_of_sight(cat.n, cat.box_len, cat.origin, cat.observer)
    rhat_c = O.line_of_sight(cat.n >> levels, cat.box_len, cat.origin, cat.observer)
    plain = O.reconstruct_field(delta, cat.box_len, cat.origin, cat.observer, cat.bias, cat.growth, n_passes=0)
    u_p = np.sum(plain["psi"] * rhat, axis=0)
    du = C.coarse_grid_correction(th.astype(np.float64), delta, u_p, rhat_c, levels, bf16_mode=True,
                                  conv_fn=C.conv_loops)
    ref = O.reconstruct_field(delta, cat.box_len, cat.origin, cat.observer, cat.bias, cat.growth,
                              n_passes=2, start=O.START_LEARNED, start_correction=du)
    e = rel_l2(psi, ref["psi"])
    print(f"n={n} network grid {n >> levels}^3: learned start psi rel L2 {e:.2e}, eps {eps[0]} vs {ref['eps']}",
          flush=True)
    assert e < 1e-4
    np.testing.assert_allclose(eps[0], ref["eps"], rtol=1e-3, atol=1e-5)


def _plain_reference(native, cat, tol):
    plan = native.plan_for(cat)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve(native.START_PLAIN)
    rc, iters, eps = plan.iterate(40, tol)
    psi = plan.psi()[0].cpu().numpy()
    plan.close()
    return rc, iters[0], eps[0], psi


@pytest.mark.parametrize("kind", ["nan", "garbage"])
def test_rejected_learned_start_restarts_from_plain(gpu_lib, kind):
    # the plain iteration judges the learned start (Sec. 5.1 iteration from any start): a network
    # with a NaN parameter gives a non-finite eps_1, one with huge finite weights an eps_1 above the
    # plain start's bound beta/(1 - beta); both must restart from D_s and end on the plain result
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.74, 31, 32, ran_factor=3, bias=2.0, smooth_r=20.0)
    th = params(12)
    if kind == "nan":
        th[100] = np.nan
    else:
        th *= 40.0
    tol = 1e-4
    plan = native.plan_for(cat, keep_delta=True, start_buffers=True, cnn=True)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve(native.START_LEARNED, to_dev(th))
    rc, iters, eps = plan.iterate(40, tol)
    psi = plan.psi()[0].cpu().numpy()
    restarts = plan.restarts()
    disp = plan.shift(native.GAL, gal).cpu().numpy()
    plan.close()
    rc_p, iters_p, eps_p, psi_p = _plain_reference(native, cat, tol)
    print(f"{kind} network: rc {rc}, restarts {restarts}, passes {iters[0]} (plain {iters_p}), "
          f"eps {eps[0]} (plain {eps_p})", flush=True)
    assert rc == native.RECON_RESTARTED and restarts == [1]
    assert iters[0] == iters_p
    np.testing.assert_allclose(eps[0], eps_p, rtol=1e-4, atol=1e-7)
    assert rel_l2(psi, psi_p) < 1e-6
    ref = O.reconstruct(cat.gal_pos, None, cat.ran_pos, None, cat.n, cat.box_len, cat.origin, cat.observer,
                        cat.bias, cat.growth, cat.smooth_r, cat.mask_tau, n_passes=iters_p)
    assert rel_l2(psi, ref["psi"]) < 1e-5
    assert np.abs(disp - ref["disp_g"]).max() < 1e-4


def test_rejected_learned_start_in_fixed_pass_call(gpu_lib):
    # a call that ends right after the start pass decides eps_1 from the output's transform; a
    # rejected start then returns the plain start's displacement and continues from there next call
    from paper_1504_02591_amd import native
    cat = G.lattice_box(32, 500.0, (-500.0, 250.0, 250.0), 0.74, 33, 34, ran_factor=3, bias=2.0, smooth_r=20.0)
    th = params(13)
    th[7] = np.nan
    plan = native.plan_for(cat, keep_delta=True, start_buffers=True, cnn=True)
    gal, ran = to_dev(cat.gal_pos), to_dev(cat.ran_pos)
    plan.paint(native.GAL, gal)
    plan.paint(native.RAN, ran)
    plan.solve(native.START_LEARNED, to_dev(th))
    rc, iters, eps = plan.iterate(1, 0.0)
    assert rc == native.RECON_RESTARTED and iters[0] == 0 and eps[0] == []
    p0 = plan.psi()[0].cpu().numpy()
    rc, iters, eps = plan.iterate(3, 0.0)
    p3 = plan.psi()[0].cpu().numpy()
    plan.close()
    assert rc == native.RECON_OK and iters[0] == 3
    plain = native.plan_for(cat)
    plain.paint(native.GAL, gal)
    plain.paint(native.RAN, ran)
    plain.solve()
    plain.iterate(0, 0.0)
    q0 = plain.psi()[0].cpu().numpy()
    rc_q, it_q, eps_q = plain.iterate(3, 0.0)
    q3 = plain.psi()[0].cpu().numpy()
    plain.close()
    assert rel_l2(p0, q0) < 1e-6 and rel_l2(p3, q3) < 1e-6
    np.testing.assert_allclose(eps[0], eps_q[0], rtol=1e-4, atol=1e-7)


def test_training_resumes_bit_identically(gpu_lib, tmp_path):
    # a run stopped after half its steps, saved (parameters, Adam moments, step, schedule length, seed)
    # and resumed from the file ends on the same parameters and moments, bit for bit, as an
    # uninterrupted run of all the steps
    from paper_1504_02591_amd import learned
    geom = dict(box_len=300.0, observer=(150.0, 150.0, 150.0), bias=2.0, growth=0.7, smooth_r=0.0,
                origin=(0.0, 0.0, 0.0))
    data = []
    for i in range(3):
        delta, u_p, target, _ = sample(32, 80 + i, 300.0, geom["observer"])
        data.append((to_dev(delta), to_dev(u_p), to_dev(target)))
    p_full, s_full, _ = learned.train(data, geom, 12, 3e-3, seed=5, half=0, log_every=100)
    p_a, s_a, _ = learned.train(data, geom, 6, 3e-3, seed=5, half=0, total=12, log_every=100)
    path = str(tmp_path / "checkpoint.npz")
    learned.save_checkpoint(path, p_a, s_a, 5)
    params, state, seed = learned.load_checkpoint(path)
    assert state["step"] == 6 and state["total"] == 12 and seed == 5
    p_b, s_b, _ = learned.train(data, geom, 6, 3e-3, seed=seed, half=0, params=params, state=state, log_every=100)
    assert np.array_equal(p_b, p_full)
    assert np.array_equal(s_b["m"], s_full["m"]) and np.array_equal(s_b["v"], s_full["v"])
    assert s_b["step"] == s_full["step"] == 12
    assert not np.array_equal(p_a, p_full)
