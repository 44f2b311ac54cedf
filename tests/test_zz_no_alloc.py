"""The load that allocates nothing (ranc_load_network_static) against the
ordinary load into a caller-provided workspace.

Two loads in a row into the library-held workspace of the device, the second
with a smaller input, each run on the same inputs as a handle loaded with
ranc_load_network; output-bus spikes of every tick, final potentials and the
five counters of every sample must be identical. The second load finds the
first one's contents in the array. Also: a second handle is refused while the
first holds the array, and a network larger than the array is refused before
anything is loaded.
"""
import ctypes

import numpy as np
import pytest

from paper_2404_16208_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_16208_amd import ranc
    return ranc


def _run_both(R, net, x, S, T, path, chunks):
    """Run the same ticks on a static-workspace handle and an ordinary one;
    returns both handles (still open) and the output spikes collected per call."""
    import torch
    got = {}
    handles = {}
    for kind in ("static", "workspace"):
        g = R.RancNet(net, S, T, path=path, static_workspace=(kind == "static"))
        assert g.path == path
        spikes = {s: [] for s in range(S)}
        t = 0
        for k, graph in chunks:
            xd = torch.from_numpy(np.ascontiguousarray(x[:, t:t + k]).view(np.int32)).cuda()
            g.run(xd, k, graph=graph)
            torch.cuda.synchronize()
            for s in range(S):
                spikes[s].append(g.spikes(s, t, t + k))
            t += k
        got[kind] = {s: np.concatenate(v) for s, v in spikes.items()}
        handles[kind] = g
    return handles, got


def _assert_same(R, handles, got, S, what):
    a, b = handles["static"], handles["workspace"]
    for s in range(S):
        assert np.array_equal(got["static"][s], got["workspace"][s]), f"{what} sample {s}: output spikes differ"
        assert np.array_equal(a.potentials(s), b.potentials(s)), f"{what} sample {s}: potentials differ"
        assert a.counters(s) == b.counters(s), f"{what} sample {s}: counters differ"


def test_static_workspace_matches_caller_workspace_twice(R):
    # first load: the 512-core MNIST-shaped net on the event-driven path, 10
    # samples, at most 4 ticks per call (66.3 MB of the 67.1 MB array), 16
    # ticks as two 4-tick per-launch calls and two 4-tick graph replays
    net1 = W.mnist_net(0)
    x1 = W.mnist_inputs(0, 10, 16)
    need = R.ranc_workspace_bytes(R.Desc(net1), 10, 4, R.RANC_PATH_SPARSE)
    assert R.RANC_STATIC_WORKSPACE_BYTES - (1 << 20) < need <= R.RANC_STATIC_WORKSPACE_BYTES, need
    h1, g1 = _run_both(R, net1, x1, 10, 4, "sparse", [(4, False), (4, False), (4, True), (4, True)])
    try:
        assert sum(len(v) for v in g1["static"].values()) > 0
        _assert_same(R, h1, g1, 10, "mnist512/sparse")
        # the array is held: a second static load is refused
        d = R.Desc(W.tiny_net(0))
        h = ctypes.c_void_p(0)
        st = R._lib.ranc_load_network_static(ctypes.byref(d.c), 4, 8, R.RANC_PATH_MFMA, None, ctypes.byref(h))
        assert st == R.RANC_ESTATE and not h.value, (st, R.ranc_last_error())
    finally:
        for g in h1.values():
            g.close()
    # second load, smaller: the tiny 5-core net on the MFMA path, 4 samples x 8 ticks
    net2 = W.tiny_net(0)
    x2 = W.tiny_inputs(0, S=4, T=8)
    h2, g2 = _run_both(R, net2, x2, 4, 8, "mfma", [(8, True)])
    try:
        assert sum(len(v) for v in g2["static"].values()) > 0
        _assert_same(R, h2, g2, 4, "tiny/mfma")
    finally:
        for g in h2.values():
            g.close()


def test_static_workspace_refuses_a_network_too_large(R):
    net = W.mnist_net(0)
    d = R.Desc(net)
    need = R.ranc_workspace_bytes(d, 10, 16, R.RANC_PATH_MFMA)
    assert need > R.RANC_STATIC_WORKSPACE_BYTES
    h = ctypes.c_void_p(0)
    st = R._lib.ranc_load_network_static(ctypes.byref(d.c), 10, 16, R.RANC_PATH_MFMA, None, ctypes.byref(h))
    assert st == R.RANC_ENOMEM and not h.value
    assert "library-held workspace" in R.ranc_last_error()
    # a refused load leaves the array free for the next one
    g = R.RancNet(W.tiny_net(0), 2, 4, path="plain", static_workspace=True)
    g.close()
