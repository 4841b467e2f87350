"""Learned initial guess on the GPU against the NumPy oracle: forward pass,
loss and gradients of every parameter (BF16 storage and matrix-core sums
against the oracle rounding at the same points, and against plain FP64),
Adam step, node prediction, training on loop-generated pairs, use in the
loop with the true-residual fallback, and what the trained network gains."""
import numpy as np
import pytest

import workloads as W
from oracle import solvers, unet
from tests.gpu_util import dev, host, rel_l2, require_gpu

pytestmark = pytest.mark.gpu

# (grid, channels): the 4-level 16/32/64/64 network of the 128^3 workload on a
# 16^3 grid (levels 16, 8, 4, 2), and a non-cubic 3-level grid whose channel
# counts exercise every output-tile split of the convolution kernels
CASES = [((16, 16, 16, 4), (16, 32, 64, 64)), ((32, 16, 16, 3), (16, 32, 48))]
IDS = ["16cube-16.32.64.64", "32x16x16-16.32.48"]

# Error bounds. Against the oracle that rounds to BF16 where the GPU stores
# BF16, the remaining differences are FP32 against FP64 sums inside the
# convolutions (~1e-7 relative) and the stored values that those differences
# push across a BF16 rounding boundary: each such value moves by one BF16
# unit (2^-8 relative) and the change propagates through the later layers
# (measured on MI355X: output 9.4e-4 / 6.3e-3, worst layer gradient 1.5e-2,
# at the two grids below). Against plain FP64 the BF16 storage itself (2^-9
# relative per stored value, over ~15 layers) is the error (measured: output
# 7.0e-3 / 1.3e-2, worst layer gradient 8.4e-2, that of a level-2 layer over
# 4^3 voxels). A wrong tap, channel or mask gives errors of order one.
TOL_EMU_OUT, TOL_EMU_GRAD = 1.5e-2, 4e-2
TOL_F64_OUT, TOL_F64_GRAD = 4e-2, 2e-1


def make_net(prob, C):
    require_gpu()
    from paper_2210_00947_amd import mgar as M
    return M.Net(M.params_for(prob), channels=C)


def pair(prob, seed):
    """A density and a temperature of that density (oracle MGCG)."""
    x = W.random_density(prob.nelem, seed, 0.05, 1.0)
    t, _ = solvers.MgarSolver(prob, solvers.MgarParams(cg_max=200)).mgcg(x, np.zeros(prob.nnodes), 1e-8)
    return x, t


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_sizes_match_oracle_layout(case):
    (nx, ny, nz, lv), C = case
    prob = W.tiny_3d(nx, ny, nz, lv)
    n = make_net(prob, C)
    assert n.nparams == unet.param_layout(C)[1]
    assert n.cells == (nz, ny, nx)


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_forward_matches_oracle(case):
    import torch
    (nx, ny, nz, lv), C = case
    prob = W.tiny_3d(nx, ny, nz, lv)
    n = make_net(prob, C)
    theta = W.unet_init(C, seed=1)
    n.mgar_net_set_params(theta)
    x = W.random_density(prob.nelem, 2, 0.0, 1.0)
    T = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    n.mgar_net_infer(dev(x), 3.0, T)
    u = n.mgar_net_output().astype(np.float64)
    inp = unet.net_input(prob, x, W.element_source(prob))
    u16, _ = unet.forward(theta.astype(np.float64), inp, C, bf16=True)
    u64, _ = unet.forward(theta.astype(np.float64), inp, C)
    e16, e64 = rel_l2(u, u16), rel_l2(u, u64)
    print(f"forward: rel. L2 to the BF16-rounding oracle {e16:.2e}, to FP64 {e64:.2e}")
    assert e16 <= TOL_EMU_OUT and e64 <= TOL_F64_OUT
    # node prediction from the GPU's own output (FP64 on both sides)
    t_or = unet.to_nodes(prob, u, 3.0)
    assert np.abs(host(T) - t_or).max() <= 1e-13 * np.abs(t_or).max()


@pytest.mark.parametrize("case", CASES, ids=IDS)
def test_loss_and_gradients_match_oracle(case):
    (nx, ny, nz, lv), C = case
    prob = W.tiny_3d(nx, ny, nz, lv)
    n = make_net(prob, C)
    theta = W.unet_init(C, seed=3)
    n.mgar_net_set_params(theta)
    x, t = pair(prob, 4)
    scale = 1.1 * float(np.abs(t).max())
    loss, g = n.mgar_net_grad(dev(x), dev(t), scale)
    qe = W.element_source(prob)
    th = theta.astype(np.float64)
    loss16, g16 = unet.loss_and_grad(prob, th, x, qe, t, scale, C, bf16=True)
    loss64, g64 = unet.loss_and_grad(prob, th, x, qe, t, scale, C)
    print(f"loss {loss:.6e}, BF16-rounding oracle {loss16:.6e}, FP64 {loss64:.6e}")
    assert abs(loss - loss16) <= TOL_EMU_OUT * loss16 and abs(loss - loss64) <= TOL_F64_OUT * loss64
    lay, _ = unet.param_layout(C)
    worst = []
    for name, wo, wl, bo, co, ci, k in lay:
        for part, a, b in (("w", wo, wo + wl), ("b", bo, bo + co)):
            e16, e64 = rel_l2(g[a:b], g16[a:b]), rel_l2(g[a:b], g64[a:b])
            worst.append((e16, e64, name + part))
            assert e16 <= TOL_EMU_GRAD and e64 <= TOL_F64_GRAD, (name, part, e16, e64)
    w16, w64 = max(worst), max(worst, key=lambda v: v[1])
    print(f"gradients: worst rel. L2 to the BF16-rounding oracle {w16[0]:.2e} ({w16[2]}), "
          f"to FP64 {w64[1]:.2e} ({w64[2]})")


def test_adam_step_matches_oracle():
    """One Adam step from zero moments, given the GPU's own gradient of the
    same pair: parameters and moments equal the oracle's FP64 update stored
    in FP32."""
    prob = W.tiny_3d(16, 16, 16, 4)
    C = (16, 32, 64, 64)
    n = make_net(prob, C)
    theta = W.unet_init(C, seed=5)
    n.mgar_net_set_params(theta)
    x, t = pair(prob, 6)
    scale = float(np.abs(t).max())
    _, g = n.mgar_net_grad(dev(x), dev(t), scale)
    lr = 1e-3
    n.mgar_net_train_step(dev(x), dev(t), scale, lr)
    after = n.mgar_net_get_params().astype(np.float64)
    zero = np.zeros_like(g)
    want, _, _ = unet.adam_step(theta.astype(np.float64), zero, zero, g, 1, lr)
    # same FP64 update on both sides; the device square root may differ in
    # the last FP64 bit, which moves a stored FP32 value by at most one unit
    assert np.all(np.abs(after - want) <= 1.2e-7 * np.abs(want) + 1e-30)


def test_source_channel():
    """The third input channel follows mgar_net_set_source (source over its
    max-norm): the GPU output for the four-quadrant source matches the
    oracle's."""
    import torch
    prob = W.tiny_3d(16, 16, 16, 4)
    C = (16, 16, 16, 16)
    n = make_net(prob, C)
    theta = W.unet_init(C, seed=8)
    n.mgar_net_set_params(theta)
    qe = W.element_source(prob) * (1.0 + np.arange(prob.nelem) % 4)
    n.mgar_net_set_source(dev(qe))
    x = W.random_density(prob.nelem, 9, 0.0, 1.0)
    T = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    n.mgar_net_infer(dev(x), 1.0, T)
    u = n.mgar_net_output().astype(np.float64)
    u16, _ = unet.forward(theta.astype(np.float64), unet.net_input(prob, x, qe), C, bf16=True)
    u_uniform, _ = unet.forward(theta.astype(np.float64), unet.net_input(prob, x, W.element_source(prob)), C,
                                bf16=True)
    assert rel_l2(u, u16) <= TOL_EMU_OUT < rel_l2(u, u_uniform)


def loop_pairs(prob, maxit):
    from oracle import topopt
    xs, ts = [], []
    topopt.run_loop(prob, maxit=maxit, on_cycle=lambda k, xp, t: (xs.append(xp.copy()), ts.append(t.copy())))
    return xs, ts


def test_training_reduces_loss_on_loop_pairs():
    """Pairs from the first cycles of the optimisation loop (each scaled by
    the previous temperature's max-norm); Adam steps over them lower the loss
    on a held-out later pair."""
    prob = W.tiny_3d(32, 32, 32, 4)
    C = (16, 32, 64, 64)
    xs, ts = loop_pairs(prob, 14)
    n = make_net(prob, C)
    n.mgar_net_set_params(W.unet_init(C, seed=7))
    held_x, held_t, held_s = xs[-1], ts[-1], float(np.abs(ts[-2]).max())
    pairs = [(dev(xs[k]), dev(ts[k]), float(np.abs(ts[k - 1]).max())) for k in range(1, len(xs) - 1)]
    l0, _ = n.mgar_net_grad(dev(held_x), dev(held_t), held_s)
    for step in range(120):
        xp, tp, sc = pairs[step % len(pairs)]
        n.mgar_net_train_step(xp, tp, sc, 1e-3, want_loss=False)
    l1, _ = n.mgar_net_grad(dev(held_x), dev(held_t), held_s)
    print(f"held-out loss {l0:.3e} -> {l1:.3e}")
    assert l1 < 0.1 * l0


SEED_CFG = {"channels": (16, 32, 64, 64), "train_until": 8, "steps": 60, "lr": 1e-3}


@pytest.mark.parametrize("lag", [0, 3], ids=["foreground", "background"])
def test_learned_guess_in_the_loop_fallback(lag):
    """The loop with the learned guess (trained on cycles 2..8, evaluated from
    9 + lag; with lag > 0 the training runs on the network's own stream beside
    the solves of cycles 9 .. 8 + lag) against the plain loop: a guess is used
    only when its true residual is below that of the previous temperature,
    and every cycle's result stays within the solve tolerance of the plain
    loop's."""
    require_gpu()
    from paper_2210_00947_amd.topopt import TopOpt
    prob = W.tiny_3d(32, 32, 32, 4, maxit=16)
    plain = TopOpt(prob, W.element_source(prob), autotune=False).run(16)
    seeded_opt = TopOpt(prob, W.element_source(prob), autotune=False,
                        seed=dict(SEED_CFG, backoff=False, lag=lag))
    seeded = seeded_opt.run(16)
    late = [c for c in seeded if c.cycle > 8 + lag]
    for c in seeded:
        if 8 < c.cycle <= 8 + lag:
            assert not c.seed_used and np.isnan(c.res_seed)
    for c in late:
        assert np.isfinite(c.res_seed) and np.isfinite(c.res_prev)
        assert c.seed_used == (c.res_seed < c.res_prev)
    for a, b in zip(plain, seeded):
        assert abs(a.compliance - b.compliance) <= 1e-6 * abs(a.compliance)
    its_plain = np.mean([c.cg_iters for c in plain if c.cycle > 8 + lag])
    its_seed = np.mean([c.cg_iters for c in late])
    ratio = np.median([c.res_seed / c.res_prev for c in late])
    print(f"learned guess in the loop: used in {sum(c.seed_used for c in late)}/{len(late)} cycles; median "
          f"residual ratio guess/previous {ratio:.3g}; mean CG iterations {its_seed:.2f} vs {its_plain:.2f} plain")
    # outcome (MI355X: ratio ~95, never used): the previous temperature of a
    # slowly changing design is a far better start than the network's guess,
    # and the fallback leaves the iterations of the plain loop
    assert ratio > 1.0 and its_seed == its_plain


def test_background_training_gives_the_foreground_parameters():
    """Training on the network's own stream beside the solves (lag > 0) runs
    the same steps on the same pairs as training in the foreground: the
    parameters agree bit for bit."""
    require_gpu()
    from paper_2210_00947_amd.topopt import TopOpt
    prob = W.tiny_3d(32, 32, 32, 4, maxit=16)
    thetas = []
    for lag in (0, 2):
        opt = TopOpt(prob, W.element_source(prob), autotune=False,
                     seed=dict(SEED_CFG, train_until=6, steps=30, lag=lag))
        opt.run(10)
        thetas.append(opt.net.mgar_net_get_params())
    assert np.array_equal(thetas[0], thetas[1])


def test_cold_start_gain_on_a_held_out_design():
    """What the trained network gains where no previous temperature exists
    (the first solve of a new design): trained on the pairs of the first loop
    cycles, its guess for a held-out later design against T0 = 0. Outcome
    (MI355X: error 0.14, residual 80 ||q||, 14 against 12 iterations): the
    guess is within 25 % of the solution, but its error is rough at the
    element scale, so its true residual exceeds ||q|| (that of T0 = 0) and
    MGCG to a relative residual of 1e-8 needs no fewer iterations from it. In
    the loop the true-residual test therefore keeps the previous temperature
    (test_learned_guess_in_the_loop_fallback)."""
    import torch
    from paper_2210_00947_amd import mgar as M
    prob = W.tiny_3d(32, 32, 32, 4)
    C = (16, 32, 64, 64)
    xs, ts = loop_pairs(prob, 14)
    n = make_net(prob, C)
    n.mgar_net_set_params(W.unet_init(C, seed=7))
    pairs = [(dev(xs[k]), dev(ts[k]), float(np.abs(ts[k - 1]).max())) for k in range(1, len(xs) - 1)]
    for step in range(120):
        xp, tp, sc = pairs[step % len(pairs)]
        n.mgar_net_train_step(xp, tp, sc, 1e-3, want_loss=False)
    x, scale = dev(xs[-1]), float(np.abs(ts[-2]).max())
    h = M.Handle(M.params_for(prob))
    q = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    h.mgar_load_vector(dev(W.element_source(prob)), q)
    guess = torch.empty(prob.nnodes, dtype=torch.float64, device="cuda")
    n.mgar_net_infer(x, scale, guess)
    r_guess = h.mgar_residual(x, q, guess)
    T = torch.empty_like(guess)
    its0 = h.mgcg_solve(x, q, None, 1e-8, T)["cg_iters"]
    its1 = h.mgcg_solve(x, q, guess, 1e-8, T)["cg_iters"]
    e_guess = rel_l2(host(guess), host(T))
    print(f"cold start on a held-out design: relative error of the guess {e_guess:.3g}, relative residual "
          f"{r_guess:.3g} (1 for T0 = 0); MGCG iterations {its1} from the guess vs {its0} from zero")
    assert e_guess < 0.25
    assert r_guess > 1.0 and its1 >= its0
