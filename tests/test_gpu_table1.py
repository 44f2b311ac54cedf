"""GPU parity on the paper's Table I workload shapes that need no trained
network: the TrueNorth reference (4096 cores of 256 x 256, 500 ticks, no
input: the engine's fixed cost, no neuron ever spikes) and the VMM
applications (21 cores of 256 x 256 for 788 ticks; 45 and 51 cores of
512 axons x 256 neurons for 889 and 1095 ticks), one instance each, at the
table's full tick counts, in graph-replayed 128-tick calls as the benchmark
runs them; every output-bus spike of every tick, the final potentials and the
counters against the oracle, on all three paths.
"""
import numpy as np
import pytest

from oracle import ranc_oracle as O
from paper_2404_16208_amd import workloads as W
from tests.parity_utils import log

pytestmark = pytest.mark.gpu

APPS = ["TrueNorth Ref.", "VMM 32x32", "VMM 50x50", "VMM 60x60"]
RT = 128


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_16208_amd import ranc  # noqa: F401


_refs = {}


def _oracle(name):
    if name not in _refs:
        T = [r[1] for r in W.TABLE1 if r[0] == name][0]
        net = W.table1_net(name)
        x = W.table1_inputs(name, net, 1, T)
        log(f"[table1] oracle: {name}, {net.num_cores} cores, {T} ticks")
        _refs[name] = (net, x, T, O.simulate(net, x, T)[0])
    return _refs[name]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("path", ["plain", "mfma", "sparse"])
@pytest.mark.parametrize("name", APPS)
def test_table1_shape_against_oracle(name, path):
    import torch
    from paper_2404_16208_amd.ranc import RancNet
    net, x, T, ref = _oracle(name)
    g = RancNet(net, 1, RT, path=path)
    got = []
    bufs = {}
    for t0 in range(0, T, RT):
        k = min(RT, T - t0)
        xd = None
        if x is not None:
            xd = bufs.setdefault(k, torch.empty((1, k) + x.shape[2:], dtype=torch.int32, device="cuda"))
            xd.copy_(torch.from_numpy(np.ascontiguousarray(x[:, t0:t0 + k]).view(np.int32)))
        g.run(xd, k, graph=True)
        got.append(g.spikes(0, t0, t0 + k))
    ev = np.concatenate(got)
    assert np.array_equal(ev, ref["events"]), f"{name}/{path}: {len(ev)} vs {len(ref['events'])} output spikes"
    assert np.array_equal(g.potentials(0), ref["v"]), f"{name}/{path}: potentials differ"
    c = g.counters(0)
    assert all(c[k] == ref["counters"][k] for k in c), (name, path, c, ref["counters"])
    if name.startswith("TrueNorth"):
        assert ref["counters"]["emitted"] == 0
    else:
        assert ref["counters"]["emitted"] > 0 and len(ref["events"]) > 0
    g.close()
