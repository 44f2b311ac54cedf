"""GPU tests of the state-resident tick loop (RANC_RUN_RESIDENT): one
persistent cooperative launch per call that keeps each 64-sample group's
potentials in LDS across the call's ticks. Results are compared with the
oracle element by element (every output-bus spike, final potentials,
counters) for every sample, including ragged sample counts, more cores than
workgroups (two cores per workgroup), the neuron-model options, calls mixed
with the per-tick forms on one handle, and the bounded-wait give-up path
(forced from the host with a zero wait limit: every workgroup still exits
normally)."""
import numpy as np
import pytest

from paper_2404_16208_amd import workloads as W
from tests.parity_utils import assert_sample_equal, log, oracle_results

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_16208_amd import ranc  # noqa: F401  (fails loudly if the library is missing)


def _run(g, x, chunks, modes):
    """Advance g call by call; modes[i] in {"resident", "graph", "eager"}."""
    import torch
    t0 = 0
    xd = torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).cuda() if x is not None else None
    for k, mode in zip(chunks, modes):
        xi = xd[:, t0:t0 + k].contiguous() if xd is not None else None
        g.run(xi, k, graph=mode == "graph", resident=mode == "resident")
        t0 += k
    torch.cuda.synchronize()
    return t0


RES_SHAPES = [
    # C, A, weight_bits, potential_bits, max_delay, grid_w, S, chunks, extra
    (6, 256, 9, 32, 4, 3, 70, [5, 7], {}),
    (5, 128, 9, 16, 3, 5, 64, [6, 6], {}),
    (4, 64, 8, 32, 2, 2, 130, [4, 4, 4], {}),
    (3, 256, 8, 12, 7, 3, 1, [9, 3], {}),
    (4, 256, 9, 32, 5, 2, 65, [8], dict(floor_range=(-40, -1), linear_frac=0.5, leak_bits=6, reset_bits=5)),
    (2, 128, 6, 10, 15, 2, 66, [16, 4], dict(floor_range=(-200, -1), linear_frac=0.3)),
    # more cores than the grid has workgroups on a 256-CU device: two per workgroup
    (300, 256, 9, 32, 4, 20, 64, [3, 3], {}),
]


@pytest.mark.parametrize("shape", RES_SHAPES, ids=lambda s: "C{}A{}b{}P{}D{}S{}".format(s[0], s[1], s[2], s[3],
                                                                                         s[4], s[6]))
def test_resident_against_oracle(shape):
    from paper_2404_16208_amd.ranc import RancNet
    C, A, b, P, D, gw, S, chunks, extra = shape
    net = W.random_net(500 + C + A + S, C, A, 256, 4, weight_bits=b, potential_bits=P, max_delay=D, grid_w=gw,
                       density=0.25, p_core=0.85, p_out=0.1, thr_range=(40, 300), config_id=870, **extra)
    T = sum(chunks)
    x = W.bernoulli_inputs(7, net, S, T, 0.15, config_id=870)
    g = RancNet(net, S, max(chunks), path="mfma")
    log(f"[resident] C={C} A={A} b={b} P={P} S={S} chunks={chunks}")
    _run(g, x, chunks, ["resident"] * len(chunks))
    assert g.tick == T
    ref = oracle_results(net, x, T, range(S))
    for s in range(S):
        assert_sample_equal(g, ref[s], s, T, what=f"resident C{C}A{A}")
    g.close()


def test_resident_mixed_with_per_tick_forms():
    """One handle advanced by resident, eager and graph calls in turn equals
    the oracle (the resident loop keeps the per-tick loop's state layout)."""
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(611, 6, 256, 256, 4, weight_bits=9, max_delay=4, grid_w=3, density=0.25, p_core=0.85,
                       p_out=0.1, thr_range=(40, 300), config_id=871)
    chunks, modes = [4, 6, 3, 5, 4], ["resident", "eager", "resident", "graph", "resident"]
    T = sum(chunks)
    x = W.bernoulli_inputs(8, net, 70, T, 0.15, config_id=871)
    g = RancNet(net, 70, 6, path="mfma")
    _run(g, x, chunks, modes)
    ref = oracle_results(net, x, T, range(70))
    for s in range(70):
        assert_sample_equal(g, ref[s], s, T, what="resident mixed")
    g.close()


def test_resident_profile_counts_launches():
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(612, 4, 128, 256, 2, weight_bits=8, grid_w=2, config_id=872)
    x = W.bernoulli_inputs(9, net, 64, 12, 0.1, config_id=872)
    g = RancNet(net, 64, 4, path="mfma")
    g.profile(True)
    _run(g, x, [4, 4, 4], ["resident"] * 3)
    p = g.profile_read()
    g.profile(False)
    assert p["resident_launches"] == 3 and p["resident_ms"] > 0
    assert p["integrate_launches"] == 0 and p["graph_launches"] == 0
    g.close()


def test_resident_gives_up_and_recovers(monkeypatch):
    """A zero wait limit makes the first grid barrier give up (forced from the
    host: every workgroup sees the flag and leaves the kernel normally); the
    call returns RANC_ETIMEOUT, later runs RANC_ESTATE until the state is
    reset, and a rerun from the reset state equals the oracle."""
    from paper_2404_16208_amd import ranc as R
    net = W.random_net(613, 6, 256, 256, 4, weight_bits=9, grid_w=3, density=0.25, thr_range=(40, 300),
                       config_id=873)
    x = W.bernoulli_inputs(10, net, 64, 8, 0.15, config_id=873)
    g = R.RancNet(net, 64, 8, path="mfma")
    monkeypatch.setenv("RANC_RESIDENT_WAIT_US", "0")
    with pytest.raises(R.RancError) as e:
        _run(g, x, [8], ["resident"])
    assert e.value.status == R.RANC_ETIMEOUT
    monkeypatch.delenv("RANC_RESIDENT_WAIT_US")
    with pytest.raises(R.RancError) as e:
        _run(g, x, [8], ["eager"])
    assert e.value.status == R.RANC_ESTATE
    g.reset()
    _run(g, x, [8], ["resident"])
    ref = oracle_results(net, x, 8, range(64))
    for s in range(64):
        assert_sample_equal(g, ref[s], s, 8, what="resident after give-up")
    g.close()


def test_resident_refuses_what_it_cannot_run():
    import torch
    from paper_2404_16208_amd import ranc as R
    x = None
    cases = [
        ("plain path", W.random_net(614, 4, 256, 256, 4, grid_w=2, config_id=874), "plain", False),
        ("128-neuron cores", W.random_net(615, 4, 256, 128, 4, grid_w=2, config_id=874), "mfma", False),
        ("512 axons", W.random_net(616, 2, 512, 256, 4, weight_bits=8, grid_w=2, config_id=874), "mfma", False),
        ("link counting", W.random_net(617, 4, 256, 256, 4, grid_w=2, config_id=874), "mfma", True),
    ]
    for what, net, path, links in cases:
        g = R.RancNet(net, 8, 4, path=path)
        if links:
            g.count_links(True)
        with pytest.raises(R.RancError) as e:
            g.run(x, 4, resident=True)
        assert e.value.status == R.RANC_EUNSUPPORTED, what
        assert g.tick == 0, what   # nothing was queued
        g.run(x, 4)                # the handle still runs per tick
        torch.cuda.synchronize()
        g.close()


def test_resident_host_inputs_and_library_workspace():
    """Host inputs (staged by the library) and a handle in the library-held
    workspace run the state-resident loop too; every sample against the
    oracle over two calls."""
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(618, 6, 256, 256, 4, weight_bits=9, max_delay=3, grid_w=3, density=0.25, p_core=0.85,
                       p_out=0.1, thr_range=(40, 300), config_id=875)
    x = W.bernoulli_inputs(13, net, 70, 10, 0.15, config_id=875)
    g = RancNet(net, 70, 5, path="mfma", static_workspace=True)
    for t0 in (0, 5):
        g.run(np.ascontiguousarray(x[:, t0:t0 + 5]), 5, resident=True)
    ref = oracle_results(net, x, 10, range(70))
    for s in range(70):
        assert_sample_equal(g, ref[s], s, 10, what="resident, host inputs, library workspace")
    g.close()


def test_resident_ignores_graph_flag():
    """RANC_RUN_RESIDENT with RANC_RUN_GRAPH runs the state-resident launch
    (one launch per call already) and captures nothing."""
    from paper_2404_16208_amd.ranc import RancNet
    net = W.random_net(619, 4, 128, 256, 2, weight_bits=8, grid_w=2, density=0.25, thr_range=(40, 300),
                       config_id=876)
    x = W.bernoulli_inputs(14, net, 64, 8, 0.15, config_id=876)
    g = RancNet(net, 64, 4, path="mfma")
    g.profile(True)
    import torch
    xd = torch.from_numpy(np.ascontiguousarray(x).view(np.int32)).cuda()
    for t0 in (0, 4):
        g.run(xd[:, t0:t0 + 4].contiguous(), 4, graph=True, resident=True)
    p = g.profile_read()
    g.profile(False)
    assert p["resident_launches"] == 2 and p["graph_launches"] == 0 and p["graphs_held"] == 0
    ref = oracle_results(net, x, 8, range(64))
    for s in range(64):
        assert_sample_equal(g, ref[s], s, 8, what="resident with the graph flag")
    g.close()
