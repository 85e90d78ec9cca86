"""GPU tests of the learned CG aid (an addition to the paper's method, which
solves Eq. (7) by plain CG): the network's inference forms and its training
gradient against the FP64 oracle network, the learned solve against the
oracle's field solve, the plain-CG fallback, and the gain of the trained
network in CG iterations."""
import sys

import numpy as np
import pytest

import oracle
from oracle import convnet as ocn
from pic_cases import Case, relerr

pytestmark = pytest.mark.gpu

U_BF16 = 2.0 ** -8   # unit roundoff of bfloat16 (8 significant bits)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _split(w):
    """FP32 weight vector -> oracle layout [W1, W2, W3] in FP64."""
    w = np.asarray(w, np.float64)
    C = ocn.C
    W1 = w[:C * 9].reshape(C, 1, 3, 3)
    W2 = w[C * 9:C * 9 + C * C * 9].reshape(C, C, 3, 3)
    W3 = w[C * 9 + C * C * 9:].reshape(1, C, 3, 3)
    return [W1, W2, W3]


def _join(W):
    return np.concatenate([a.ravel() for a in W]).astype(np.float32)


def _random_weights(seed, noise=0.2):
    rng = np.random.default_rng(seed)
    return _join(ocn.init_identity(rng, noise=noise))


def _learned_sim(case, precision="fp64", **opt):
    return case.gpu_sim(precision, solver="learned", **opt)


@pytest.fixture(scope="module")
def net_sim():
    case = Case(40, 36, 1, ppc=1, gamma0=2.0, seed=0)
    sim = _learned_sim(case)
    yield sim
    sim.close()


# (ny, nx): several 16/32 tiles with ragged tails, a single partial tile, and
# a grid narrower than the 7-cell receptive field (multiple periodic wraps)
SHAPES = [(36, 40), (9, 13), (5, 4)]


@pytest.mark.parametrize("shape", SHAPES)
def test_collapsed_filter_equals_network(net_sim, shape):
    _say(f"collapsed filter vs oracle network, shape={shape}")
    w = _random_weights(1)
    net_sim.set_weights(w)
    x = np.random.default_rng(2).standard_normal(shape)
    y = net_sim.precond_apply(x, form="collapsed")
    y_ref, _ = ocn.forward(_split(w), x)
    # FP64 composition and FP64 filter against the FP64 three-layer network
    assert relerr(y, y_ref) <= 1e-12


@pytest.mark.parametrize("shape", SHAPES)
def test_mfma_network_within_bf16_bound(net_sim, shape):
    _say(f"BF16 MFMA network vs oracle network, shape={shape}")
    w = _random_weights(3)
    net_sim.set_weights(w)
    x = np.random.default_rng(4).standard_normal(shape)
    y = net_sim.precond_apply(x, form="mfma")
    W = _split(w)
    y_ref, _ = ocn.forward(W, x)
    # three roundings to bfloat16 (layer-1 output, W2, layer-2 output), each
    # bounded by U_BF16 times the magnitude network |N|(|x|); FP32 accumulation
    # adds far less
    mag, _ = ocn.forward([np.abs(a) for a in W], np.abs(x))
    bound = 3.5 * U_BF16 * mag + 1e-6 * mag.max()
    err = np.abs(y - y_ref)
    assert np.all(err <= bound), float((err / bound).max())
    assert relerr(y, y_ref) > 0.0   # BF16 is really in the loop


# whole field; windows wrapping in both directions, one cell, and a window
# as large as the field (training windows: a crop plus a 3-cell halo)
WINDOWS = [None, (35, 30, 16, 12), (3, 4, 1, 1), (0, 0, 40, 36), (7, 2, 33, 5)]


@pytest.mark.parametrize("window", WINDOWS)
def test_gradient_matches_oracle(net_sim, window):
    _say(f"training gradient vs oracle, window {window}")
    w = _random_weights(5, noise=0.1)
    net_sim.set_weights(w)
    rng = np.random.default_rng(6)
    b = rng.standard_normal((36, 40))
    t = rng.standard_normal((36, 40))
    loss, g = net_sim.precond_grad(b, t, window=window)
    L_ref, G_ref = ocn.loss_and_grad(_split(w), b, t, window=window)
    assert abs(loss - L_ref) <= 1e-5 * abs(L_ref)
    # FP32 forward/backward against FP64: layer by layer, normwise
    G = _split(g)
    for k in range(3):
        e = np.linalg.norm(G[k] - G_ref[k]) / np.linalg.norm(G_ref[k])
        assert e <= 1e-4, (k, e)


def test_apply_rejects_bad_sizes(net_sim):
    import paper_1412_2480_amd as pic
    with pytest.raises(pic.PicError):
        net_sim.precond_apply(np.zeros((2, 40)))
    with pytest.raises(pic.PicError):
        net_sim.precond_apply(np.zeros((40, 40)))   # more cells than run 0 holds
    with pytest.raises(pic.PicError):
        net_sim.set_weights(np.zeros(10, np.float32))
    z = np.zeros((36, 40))
    for win in ((40, 0, 4, 4), (0, -1, 4, 4), (0, 0, 41, 4), (0, 0, 4, 0)):
        with pytest.raises(pic.PicError):
            net_sim.precond_grad(z, z, window=win)


def test_precond_calls_need_learned_solver():
    import paper_1412_2480_amd as pic
    case = Case(24, 20, 1, ppc=1, gamma0=2.0, seed=0)
    sim = case.gpu_sim("fp64")
    with pytest.raises(pic.PicError) as e:
        sim.precond_use(True)
    assert e.value.code == -7
    sim.close()


def _dB_after_split_step(sim, case):
    sim.gather_push()
    sim.deposit()
    st = sim.field_solve()
    dB = [sim.get_field(0, n) - case.fields[n] for n in ("Bx", "By", "Bz")]
    return st, dB


@pytest.mark.parametrize("form", ["collapsed", "mfma"])
def test_learned_solve_matches_oracle(form):
    _say(f"learned solve vs oracle, form={form}")
    case = Case(40, 36, 2, ppc=3, gamma0=5.0, T=0.05, field_amp=0.5, seed=7)
    ref = case.oracle_sim(rtol=1e-14)
    ref.push_deposit()
    B0 = [b.copy() for b in ref.B]
    ref.field_solve()
    dB_ref = [ref.B[k] - B0[k] for k in range(3)]
    sim = _learned_sim(case, learned_form=form)
    sim.set_weights(_random_weights(8, noise=0.05))
    st, dB = _dB_after_split_step(sim, case)
    s = st[0]
    assert s["fallback"] == 0
    for c in range(3):
        assert s["relres"][c] <= case.rtol
        assert s["learned_iters"][c] >= 1
        # residual 1e-8 and cond(A) < 4 bound the solution error by ~4e-8
        assert relerr(dB[c], dB_ref[c]) <= 1e-6, c
    sim.close()


def test_fallback_to_plain_cg():
    _say("learned budget 1 -> plain CG finishes")
    case = Case(40, 36, 2, ppc=3, gamma0=5.0, T=0.05, field_amp=0.5, seed=9)
    sim = _learned_sim(case, learned_maxit=1)
    st, _ = _dB_after_split_step(sim, case)
    s = st[0]
    assert s["fallback"] == 1
    for c in range(3):
        assert s["learned_iters"][c] == 1
        assert s["iters"][c] > 1
        assert s["relres"][c] <= case.rtol
    sim.close()


def test_training_gain():
    """Collect (b, dB) pairs from a pair-plasma run, train on the GPU, and
    compare CG iterations with and without the network on later steps."""
    _say("learned gain: collect, train, compare")
    case = Case(128, 64, 2, ppc=8, gamma0=20.0, T=0.01, seed=11)
    sim = _learned_sim(case, precision="fp32", precond_slots=12)
    sim.precond_use(False)
    sim.precond_collect(True)
    sim.step(12)
    n_pairs = sim.precond_collect(False)
    assert n_pairs == 12
    tr = sim.precond_train(epochs=25, lr=1e-3)
    _say(f"training: {tr}")
    assert tr["samples"] == 36 and tr["updates"] == 25 * 36
    assert tr["loss_last"] < 0.05 * tr["loss_first"]
    # later steps alternate between plain CG and the learned solver
    it_plain, it_learned = [], []
    for k in range(4):
        sim.precond_use(False)
        st = sim.step(1)[0]
        it_plain.append(sum(st["iters"]))
        assert st["learned_iters"] == [0, 0, 0]
        sim.precond_use(True)
        st = sim.step(1)[0]
        it_learned.append(sum(st["iters"]))
        assert st["fallback"] == 0
        assert max(st["relres"]) <= case.rtol
    _say(f"iterations plain {it_plain} learned {it_learned}")
    assert max(it_learned) * 2 <= min(it_plain)
    sim.close()
