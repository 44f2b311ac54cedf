"""GPU parity of the packets per mesh link (Sec. III-D, Fig. 2: x first, then
y, one link per hop) against the oracle's hop-by-hop router.

Every test compares, for every listed sample, the library's per-core,
per-direction counts with the oracle's, element by element, and their sum
with the oracle's hop counter. Meshes are wide, tall, square and a single row
or column; sample counts span one and several 64-sample words with a ragged
end; runs are split into calls (and graph replays) of uneven length.
"""
import numpy as np
import pytest

from oracle import ranc_oracle as O
from paper_2404_16208_amd import workloads as W
from tests.parity_utils import log

pytestmark = pytest.mark.gpu

PATHS = ["plain", "mfma", "sparse"]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2404_16208_amd import ranc  # noqa: F401


def _run(net, x, S, chunks, path, graph, enable_at=0):
    """Run the library in calls of the given lengths; link counting is on from
    tick enable_at (a call boundary)."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet
    g = RancNet(net, S, max(chunks), path=path)
    t = 0
    for k in chunks:
        if t == enable_at:
            g.count_links(True)
        xd = torch.from_numpy(np.ascontiguousarray(x[:, t:t + k]).view(np.int32)).cuda()
        g.run(xd, k, graph=graph)
        t += k
    torch.cuda.synchronize()
    return g


def _oracle_links(net, x, T, samples, t_from=0):
    """Per sample: links counted over ticks [t_from, T), and the hop counter."""
    out = {}
    for s in samples:
        sim = O.OracleSim(net)
        if t_from:
            sim.run(x[s, :t_from], t_from)
        l0, h0 = sim.links(), sim.counters()["hops"]
        sim.run(x[s, t_from:T], T - t_from)
        out[s] = (sim.links() - l0, sim.counters()["hops"] - h0)
    return out


def _check(g, ref, what):
    for s, (links, hops) in ref.items():
        got = g.links(s)
        if not np.array_equal(got, links):
            bad = np.argwhere(got != links)
            c, d = bad[0]
            raise AssertionError(f"{what} sample {s}: {len(bad)} link counts differ, first (core {c}, dir {d}): "
                                 f"gpu {got[c, d]} oracle {links[c, d]}")
        assert int(got.sum()) == hops, f"{what} sample {s}: hops {int(got.sum())} vs {hops}"


MESHES = [  # (C, grid_w, A, N, max_delay)
    (12, 4, 64, 64, 3),
    (12, 3, 128, 64, 4),
    (16, 16, 64, 128, 2),     # one row
    (8, 1, 64, 64, 5),        # one column
    (36, 6, 256, 256, 7),
    (20, 5, 64, 512, 15),
]


@pytest.mark.parametrize("path", PATHS)
@pytest.mark.parametrize("mesh", MESHES, ids=lambda m: f"C{m[0]}w{m[1]}A{m[2]}N{m[3]}D{m[4]}")
def test_links_match_oracle(mesh, path):
    C, gw, A, N, D = mesh
    S, T = 70, 12
    net = W.random_net(40 + C + A + N, C, A, N, 4, grid_w=gw, max_delay=D, density=0.3, p_core=0.85, p_out=0.1,
                       thr_range=(32, 200), config_id=820)
    x = W.bernoulli_inputs(5, net, S, T, 0.15, config_id=820)
    log(f"[links] {net.name} mesh {gw}x{C // gw} path={path}")
    g = _run(net, x, S, [5, 7], path, graph=False)
    ref = _oracle_links(net, x, T, [0, 1, 33, 63, 64, 69])
    assert any(r[1] > 0 for r in ref.values())
    _check(g, ref, f"{net.name}/{path}")
    g.close()


@pytest.mark.parametrize("path", PATHS)
def test_links_graph_replay_and_late_enable(path):
    """Counting switched on at tick 4, then graph replays; the counts cover
    ticks 4..15 only."""
    net = W.random_net(77, 24, 128, 128, 4, grid_w=6, max_delay=6, density=0.25, p_core=0.9, p_out=0.05,
                       thr_range=(32, 160), config_id=821)
    S, T = 64, 16
    x = W.bernoulli_inputs(6, net, S, T, 0.12, config_id=821)
    g = _run(net, x, S, [4, 4, 4, 4], path, graph=True, enable_at=4)
    _check(g, _oracle_links(net, x, T, [0, 17, 63], t_from=4), f"late-enable/{path}")
    g.reset()
    import torch
    torch.cuda.synchronize()
    assert not g.links(0).any(), "reset must clear the link counts"
    g.close()


@pytest.mark.parametrize("persistent", [False, True], ids=["per_class", "persistent"])
def test_links_in_a_batch(persistent):
    """Two networks with counting on (one MFMA-path, one plain-path) and one
    without, advanced together."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet, run_batch
    nets = [W.random_net(90 + i, C, A, N, 4, grid_w=gw, max_delay=4, density=0.25, p_core=0.9, p_out=0.05,
                         thr_range=(32, 160), config_id=822)
            for i, (C, gw, A, N) in enumerate([(16, 4, 128, 256), (12, 3, 64, 64), (8, 2, 64, 128)])]
    S, T = 64, 10
    xs = [W.bernoulli_inputs(7 + i, n, S, T, 0.12, config_id=822) for i, n in enumerate(nets)]
    gs = [RancNet(nets[0], S, T, path="mfma"), RancNet(nets[1], S, T, path="plain"),
          RancNet(nets[2], S, T, path="mfma")]
    gs[0].count_links(True)
    gs[1].count_links(True)
    xd = [torch.from_numpy(x.view(np.int32)).cuda() for x in xs]
    run_batch(gs, xd, T, graph=True, persistent=persistent)
    torch.cuda.synchronize()
    for i in (0, 1):
        _check(gs[i], _oracle_links(nets[i], xs[i], T, [0, 31, 63]), f"batch net {i}")
    assert not gs[2].links(0).any()
    for g in gs:
        g.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("path", ["sparse", "mfma"])
def test_links_on_the_16384_core_mesh(path):
    """The 128 x 128 mesh with random destinations, 64 samples, the first 20
    ticks in two graph-replayed calls; samples 0, 21 and 63 against the oracle."""
    import torch
    from paper_2404_16208_amd.ranc import RancNet
    net = W.sparse_mesh_net(0)
    S, T, TC = 64, 20, 10
    x = W.sparse_mesh_inputs(0, net, S, T)
    g = RancNet(net, S, TC, path=path)
    g.count_links(True)
    buf = torch.empty((S, TC) + x.shape[2:], dtype=torch.int32, device="cuda")
    for t0 in range(0, T, TC):
        buf.copy_(torch.from_numpy(np.ascontiguousarray(x[:, t0:t0 + TC]).view(np.int32)))
        g.run(buf, TC, graph=True)
    torch.cuda.synchronize()
    log(f"[links] mesh16384/{path}: oracle for 3 samples x {T} ticks")
    samples = [0, 21, 63]
    ref = {}
    res = O.simulate(net, x, T, samples=samples)
    for r in res:
        ref[r["sample"]] = (r["links"], r["counters"]["hops"])
    _check(g, ref, f"mesh16384/{path}")
    g.close()
