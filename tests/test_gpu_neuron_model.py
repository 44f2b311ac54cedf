"""GPU parity of the neuron-model options on every path: potential widths
below 32 bits, leak and reset widths, a floor (negative threshold) and linear
reset (Sec. I and Sec. V name the widths of weight, leak, potential and reset
as configurable). The oracle applies them in int64 in the order of its
potential update; the kernels use the saturating 32-bit form."""
import numpy as np
import pytest

from paper_2404_16208_amd import workloads as W
from tests.parity_utils import assert_parity, oracle_results, assert_sample_equal, log

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_16208_amd import ranc  # noqa: F401  (fails loudly if the library is missing)


MODEL_SHAPES = [
    # C, A, N, G, weight_bits, potential_bits, max_delay, grid_w, S, T
    (6, 256, 256, 4, 9, 32, 4, 3, 70, 12),    # two weight planes
    (4, 64, 64, 2, 4, 12, 2, 2, 70, 10),      # 64-neuron cores (dead blocks on the MFMA path)
    (3, 512, 128, 4, 9, 16, 4, 3, 70, 8),     # plane split
    (3, 256, 512, 4, 9, 20, 4, 3, 130, 8),    # two neuron slices
    (4, 128, 128, 8, 8, 32, 3, 2, 100, 9),
]
MODELS = {
    "floor": dict(floor_range=(-300, 50)),
    "linear": dict(linear_frac=0.5),
    "floor_linear": dict(floor_range=(-200, 0), linear_frac=0.5),
}


def model_net(shape, model, seed=0):
    C, A, N, G, b, P, D, gw, S, T = shape
    wmax = (1 << (b - 1)) - 1
    lim = (1 << (P - 1)) - 1
    return W.random_net(2000 + seed + C * A + N + G + b + P + D, C, A, N, G, weight_bits=b, potential_bits=P,
                        max_delay=D, grid_w=gw, density=0.25, p_core=0.7, p_out=0.25,
                        leak_range=(-6, 4), thr_range=(max(1, wmax // 2), min(lim, 4 * wmax)),
                        reset_range=(-3, 2), vinit_range=(-5, 5), input_cores=list(range(0, C, 2)),
                        config_id=710, leak_bits=5, reset_bits=4, **MODELS[model])


@pytest.mark.parametrize("model", list(MODELS))
@pytest.mark.parametrize("shape", MODEL_SHAPES, ids=lambda s: "C{}A{}N{}G{}b{}P{}D{}".format(*s[:7]))
@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
def test_neuron_model_options(shape, model, path):
    C, A, N, G, b, P, D, gw, S, T = shape
    net = model_net(shape, model)
    x = W.bernoulli_inputs(12, net, S, T, 0.3, config_id=710)
    assert_parity(net, x, T, path, what=f"{model}{shape[:7]}")


@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
@pytest.mark.parametrize("pbits", [8, 32])
def test_linear_reset_and_floor_at_range_ends(path, pbits):
    """Linear reset where U - threshold overflows int32 (threshold at the
    bottom of the range, U at the top) and floors at both range ends."""
    net = W.random_net(90 + pbits, 4, 64, 128, 2, weight_bits=9, potential_bits=pbits, max_delay=2, grid_w=2,
                       density=0.5, p_core=0.5, p_out=0.5, input_cores=[0, 1, 2, 3], config_id=711,
                       floor_range=(-1, 0), linear_frac=0.7)
    r = np.random.default_rng(pbits + 1)
    lo, hi = -(1 << (pbits - 1)), (1 << (pbits - 1)) - 1
    shape = net.v_init.shape
    net.v_init[:] = r.choice(np.array([lo, hi, lo + 1, hi - 1, 0], np.int64), size=shape)
    net.reset[:] = r.choice(np.array([lo, hi, 0], np.int64), size=shape)
    net.leak[:] = r.choice(np.array([-(1 << 30), 1 << 30, -1, 1, 0, hi, lo], np.int64)
                           .clip(-(1 << 30), 1 << 30), size=shape)
    net.threshold[:] = r.choice(np.array([2**31 - 1, -2**31, hi, lo, 0, 100], np.int64), size=shape)
    net.floor[:] = r.choice(np.array([lo, hi, lo + 1, -50, 0], np.int64), size=shape)
    x = W.bernoulli_inputs(15, net, 70, 12, 0.4, config_id=711)
    assert_parity(net, x, 12, path, what=f"model_extremes_P{pbits}")


@pytest.mark.parametrize("persistent", [False, True], ids=["per_class", "persistent"])
def test_batch_mixes_model_options(persistent):
    """Networks with and without the extended update in one batch: the
    per-class launches split them by potential update, the persistent launch
    runs both from one queue."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet, run_batch
    nets = [model_net(MODEL_SHAPES[0], "floor_linear", 1), model_net(MODEL_SHAPES[0], "floor", 2),
            W.random_net(77, 6, 256, 256, 4, grid_w=3, p_core=0.7, p_out=0.25, input_cores=[0, 2, 4],
                         config_id=712),
            model_net(MODEL_SHAPES[2], "linear", 3)]
    S, T = 70, 8
    xs = [W.bernoulli_inputs(16 + i, n, S, T, 0.3, config_id=712) for i, n in enumerate(nets)]
    gs = [RancNet(n, S, T, path="mfma") for n in nets]
    run_batch(gs, [torch.from_numpy(x.view(np.int32)).cuda() for x in xs], T, graph=True, persistent=persistent)
    torch.cuda.synchronize()
    for i, (n, x, g) in enumerate(zip(nets, xs, gs)):
        ref = oracle_results(n, x, T, [0, 33, 69])
        for s, r in ref.items():
            assert_sample_equal(g, r, s, T, what=f"batch{i}")
        g.close()
