"""Pins that tie the serial oracle to what the paper and mathematics fix.

Each ``pin_*`` function takes an optional bound oracle library (``lib``; None =
the default build) and raises AssertionError on a mismatch. They are run
against the real oracle by ``test_oracle_pins.py`` and against copies of the
oracle with deliberately planted mistakes by ``test_oracle_mutations.py``,
which checks that every planted mistake is caught by at least one pin.

What pins what:
  - hand-derived single-neuron closed forms (tests/golden/single_neuron_cases.txt)
    and a randomized closed-form sweep: integrate / leak / threshold (>=) /
    reset / saturation (GPU-RANC Sec. II, Algorithm 1 neuron loop);
  - axon-type weight selection (Sec. II: weight chosen by axon type);
  - one tick of integration against a numpy int64 matrix product
    x @ B with B[a, n] = crossbar[a, n] * W[n, type[a]] (the plain
    definition of the accumulate loop);
  - delivery tick, ring reuse, two-hop routes and boolean merge
    (tests/golden/routing_cases.txt; Sec. III-D, III-E);
  - an independent pure-Python simulator on tiny nets, random and exhaustive
    over input patterns;
  - invariants: routed/out counts against the spike trace, delivered <= routed,
    potential bounds, silence without drive, resume and prefix consistency,
    core relabeling, hop counts equal |dx| + |dy| (Sec. III-D, Fig. 2).
"""
from __future__ import annotations

import math
import os
import re

import numpy as np

from oracle import ranc_oracle as O
from paper_2404_16208_amd import workloads as W
from tests.brute_sim import brute_simulate

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


# ---------------------------------------------------------------- helpers

def parse_golden(name):
    cases, cur = {}, None
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            m = re.match(r"\[(\w+)\]$", line)
            if m:
                cur = cases.setdefault(m.group(1), {})
                continue
            k, v = [x.strip() for x in line.split("=", 1)]
            cur[k] = v
    return cases


def make_net(C, A, N, G=1, grid_w=None, conn=None, axon_type=None, weight=None, leak=0,
             threshold=1 << 30, reset=0, v_init=0, dest_kind=0, dest_dx=0, dest_dy=0,
             dest_axon=0, dest_delay=0, potential_bits=32, max_delay=4, input_cores=(0,),
             weight_bits=9, floor=None, reset_mode=None, leak_bits=32, reset_bits=32):
    grid_w = grid_w or C
    full = lambda v, shape, dt: np.broadcast_to(np.asarray(v, dtype=dt), shape).copy()
    conn = np.ones((C, A, N), bool) if conn is None else np.asarray(conn, bool)
    return W.Net(C, A, N, G, weight_bits, potential_bits, max_delay, grid_w, C // grid_w,
                 W.pack_bits(conn),
                 full(0 if axon_type is None else axon_type, (C, A), np.uint8),
                 full(0 if weight is None else weight, (C, N, G), np.int16),
                 full(leak, (C, N), np.int32), full(threshold, (C, N), np.int32),
                 full(reset, (C, N), np.int32), full(v_init, (C, N), np.int32),
                 full(dest_kind, (C, N), np.uint8), full(dest_dx, (C, N), np.int16),
                 full(dest_dy, (C, N), np.int16), full(dest_axon, (C, N), np.uint16),
                 full(dest_delay, (C, N), np.uint8),
                 np.asarray(input_cores, np.int32), leak_bits=leak_bits, reset_bits=reset_bits,
                 floor=None if floor is None else full(floor, (C, N), np.int32),
                 reset_mode=None if reset_mode is None else full(reset_mode, (C, N), np.uint8)).contiguous()


def ext_from_ticks(T, n_in, A, spikes):
    """spikes: iterable of (tick, input_index, axon)."""
    ext = np.zeros((T, n_in, (A + 31) // 32), np.uint32)
    for t, k, a in spikes:
        ext[t, k, a // 32] |= np.uint32(1 << (a % 32))
    return ext


def run1(net, ext, T, lib=None, trace=False):
    sim = O.OracleSim(net, lib)
    ev, st, vt = sim.run(ext, T, trace=trace)
    return ev, sim.potentials(), sim.counters(), st, vt, sim


def single_neuron(weight, leak, threshold, reset, v_init, potential_bits, every, T, floor=None,
                  reset_mode=None):
    net = make_net(1, 1, 1, G=1, weight=weight, leak=leak, threshold=threshold, reset=reset,
                   v_init=v_init, potential_bits=potential_bits, dest_kind=W.DEST_OUT, floor=floor,
                   reset_mode=reset_mode)
    ext = ext_from_ticks(T, 1, 1, [(t, 0, 0) for t in range(T)] if every else [])
    return net, ext


def closed_form(u, thr, reset, v0, T):
    """Spike ticks and final V for constant drive u > 0 (v0 < thr, reset < thr)."""
    t1 = math.ceil((thr - v0) / u) - 1
    p = math.ceil((thr - reset) / u)
    spikes = list(range(t1, T, p)) if t1 < T else []
    if spikes:
        vf = reset + (T - 1 - spikes[-1]) * u
    else:
        vf = v0 + T * u
    return spikes, vf


# ---------------------------------------------------------------- pins

def pin_single_neuron_cases(lib=None):
    for name, c in parse_golden("single_neuron_cases.txt").items():
        T = int(c["ticks"])
        net, ext = single_neuron(int(c["weight"]), int(c["leak"]), int(c["threshold"]),
                                 int(c["reset"]), int(c["v_init"]), int(c["potential_bits"]),
                                 c["input"] == "every", T)
        ev, v, cnt, *_ = run1(net, ext, T, lib)
        want = [int(x) for x in c["spikes"].split()]
        got = [int(t) for t in ev[:, 0]]
        assert got == want, f"{name}: spikes {got} != {want}"
        assert int(v[0, 0]) == int(c["v_final"]), f"{name}: V {int(v[0, 0])} != {c['v_final']}"
        assert cnt["out"] == len(want) and cnt["emitted"] == len(want), name


def pin_neuron_model_cases(lib=None):
    """Linear reset and the potential floor (tests/golden/neuron_model_cases.txt)."""
    for name, c in parse_golden("neuron_model_cases.txt").items():
        T = int(c["ticks"])
        mode = {"absolute": 0, "linear": 1}[c.get("reset_mode", "absolute")]
        net, ext = single_neuron(int(c["weight"]), int(c["leak"]), int(c["threshold"]),
                                 int(c["reset"]), int(c["v_init"]), int(c["potential_bits"]),
                                 c["input"] == "every", T, floor=int(c["floor"]) if "floor" in c else None,
                                 reset_mode=mode)
        ev, v, cnt, *_ = run1(net, ext, T, lib)
        want = [int(x) for x in c["spikes"].split()]
        got = [int(t) for t in ev[:, 0]]
        assert got == want, f"{name}: spikes {got} != {want}"
        assert int(v[0, 0]) == int(c["v_final"]), f"{name}: V {int(v[0, 0])} != {c['v_final']}"


def pin_linear_reset_sweep(lib=None, n=60, seed=8):
    """Linear reset under constant drive u: with 0 < u < threshold the neuron
    fires whenever v_init + (t+1) u passes a multiple of the threshold and
    ends at (v_init + T u) mod threshold; with u >= threshold it fires every
    tick and gains u - threshold per tick."""
    r = np.random.default_rng(seed)
    for i in range(n):
        w = int(r.integers(1, 256))
        leak = int(r.integers(-w + 1, 64))
        u = w + leak
        if i % 4 == 3:
            thr = int(r.integers(1, u + 1))
            v0 = int(r.integers(0, 50))
        else:
            thr = int(r.integers(u + 1, 3000))
            v0 = int(r.integers(0, thr))
        T = int(r.integers(1, 40))
        net, ext = single_neuron(w, leak, thr, 0, v0, 32, True, T, reset_mode=1)
        ev, v, *_ = run1(net, ext, T, lib)
        if u < thr:
            spikes = [t for t in range(T) if (v0 + (t + 1) * u) // thr > (v0 + t * u) // thr]
            vf = (v0 + T * u) % thr
        else:
            spikes, vf = list(range(T)), v0 + T * (u - thr)
        assert [int(t) for t in ev[:, 0]] == spikes, (w, leak, thr, v0, T)
        assert int(v[0, 0]) == vf, (w, leak, thr, v0, T, int(v[0, 0]), vf)


def pin_floor_sweep(lib=None, n=60, seed=9):
    """Negative constant drive u with a floor F <= v_init < threshold: the
    neuron never fires and ends at max(F, v_init + T u)."""
    r = np.random.default_rng(seed)
    for _ in range(n):
        w = int(r.integers(0, 100))
        leak = int(r.integers(-300, -w))
        u = w + leak
        F = int(r.integers(-5000, 1))
        thr = int(r.integers(1, 1000))
        v0 = int(r.integers(F, thr))
        T = int(r.integers(1, 40))
        net, ext = single_neuron(w, leak, thr, 0, v0, 32, True, T, floor=F)
        ev, v, *_ = run1(net, ext, T, lib)
        assert len(ev) == 0
        assert int(v[0, 0]) == max(F, v0 + T * u), (w, leak, F, thr, v0, T)


def pin_value_widths(lib=None):
    """Leaks and reset potentials are signed values of leak_bits and
    reset_bits bits, floors lie in the potential range, reset modes are 0 or
    1: the oracle rejects a description with a value just outside its range
    and accepts the values at the ends of it."""
    lib = lib if lib is not None else O._load()
    for bits in (2, 4, 9, 17):
        lo, hi = -(1 << (bits - 1)), (1 << (bits - 1)) - 1
        for v, ok in ((lo, True), (hi, True), (lo - 1, False), (hi + 1, False)):
            assert (O.check(make_net(1, 1, 2, leak=[[0, v]], leak_bits=bits), lib) == 0) == ok, ("leak", bits, v)
            assert (O.check(make_net(1, 1, 2, reset=[[0, v]], reset_bits=bits), lib) == 0) == ok, ("reset", bits, v)
    for P in (8, 12):
        lo, hi = -(1 << (P - 1)), (1 << (P - 1)) - 1
        for v, ok in ((lo, True), (hi, True), (lo - 1, False), (hi + 1, False)):
            assert (O.check(make_net(1, 1, 2, floor=[[0, v]], potential_bits=P), lib) == 0) == ok, ("floor", P, v)
    for m, ok in ((0, True), (1, True), (2, False)):
        assert (O.check(make_net(1, 1, 2, reset_mode=[[0, m]]), lib) == 0) == ok, ("reset_mode", m)
    assert O.check(make_net(1, 1, 2, leak_bits=1), lib) != 0
    assert O.check(make_net(1, 1, 2, reset_bits=33), lib) != 0


def pin_closed_form_sweep(lib=None, n=60, seed=1):
    r = np.random.default_rng(seed)
    for _ in range(n):
        w = int(r.integers(1, 256))
        leak = int(r.integers(-w + 1, 64))
        u = w + leak
        thr = int(r.integers(1, 3000))
        reset = int(r.integers(-500, thr))
        v0 = int(r.integers(-500, thr))
        T = int(r.integers(1, 40))
        net, ext = single_neuron(w, leak, thr, reset, v0, 32, True, T)
        ev, v, *_ = run1(net, ext, T, lib)
        spikes, vf = closed_form(u, thr, reset, v0, T)
        assert [int(t) for t in ev[:, 0]] == spikes, (w, leak, thr, reset, v0, T)
        assert int(v[0, 0]) == vf, (w, leak, thr, reset, v0, T, int(v[0, 0]), vf)


def pin_axon_types(lib=None):
    # 4 axons of types 0..3, weights 1, 10, 100, 1000: one tick of input on a
    # subset of axons gives the sum of the selected types' weights.
    wts = [1, 10, 100, 1000]
    for perm in ([0, 1, 2, 3], [3, 1, 0, 2], [2, 3, 1, 0]):
        for mask in range(16):
            net = make_net(1, 4, 1, G=4, axon_type=perm, weight=[[wts]])
            ext = ext_from_ticks(1, 1, 4, [(0, 0, a) for a in range(4) if mask >> a & 1])
            _, v, cnt, *_ = run1(net, ext, 1, lib)
            want = sum(wts[perm[a]] for a in range(4) if mask >> a & 1)
            assert int(v[0, 0]) == want, (perm, mask, int(v[0, 0]), want)
            assert cnt["events"] == bin(mask).count("1")


def pin_integration_matmul(lib=None, seed=2):
    r = np.random.default_rng(seed)
    for A, N, G in ((40, 70, 3), (96, 33, 4), (64, 64, 8), (7, 130, 2)):
        conn = r.random((1, A, N)) < 0.3
        typ = r.integers(0, G, size=(1, A))
        wt = r.integers(-256, 256, size=(1, N, G))
        net = make_net(1, A, N, G=G, conn=conn, axon_type=typ, weight=wt)
        x = r.random(A) < 0.5
        ext = W.pack_bits(x[None, None, :])
        _, v, cnt, *_ = run1(net, ext, 1, lib)
        B = conn[0].astype(np.int64) * wt[0][:, typ[0]].T.astype(np.int64)  # [A, N]
        want = x.astype(np.int64) @ B
        assert np.array_equal(v[0].astype(np.int64), want), (A, N, G)
        assert cnt["events"] == int(x.astype(np.int64) @ conn[0].sum(axis=1))


def _delay_net(d, max_delay=3):
    return make_net(2, 1, 1, G=1, grid_w=2, weight=10, threshold=10,
                    dest_kind=[[W.DEST_CORE], [W.DEST_OUT]], dest_dx=[[1], [0]],
                    dest_axon=0, dest_delay=[[d], [0]], max_delay=max_delay)


def _events_str(ev):
    return " ; ".join(" ".join(str(int(x)) for x in e) for e in ev)


def pin_delay_delivery(lib=None):
    g = parse_golden("routing_cases.txt")
    for d in (1, 2, 3):
        ev, *_ = run1(_delay_net(d), ext_from_ticks(8, 1, 1, [(0, 0, 0)]), 8, lib)
        assert _events_str(ev) == g[f"delay_d{d}"]["out"], (d, _events_str(ev))
    ev, *_ = run1(_delay_net(3), ext_from_ticks(10, 1, 1, [(0, 0, 0), (4, 0, 0), (5, 0, 0)]), 10, lib)
    assert _events_str(ev) == g["delay_wrap"]["out"], _events_str(ev)
    # two hops on a 2x2 mesh: core0 -> core3 (dx=1,dy=1, d=2) -> core2 (dx=-1, d=3) -> OUT
    net = make_net(4, 1, 1, G=1, grid_w=2, weight=10, threshold=10,
                   dest_kind=[[W.DEST_CORE], [W.DEST_NONE], [W.DEST_OUT], [W.DEST_CORE]],
                   dest_dx=[[1], [0], [0], [-1]], dest_dy=[[1], [0], [0], [0]],
                   dest_delay=[[2], [0], [0], [3]], max_delay=3)
    ev, _, cnt, _, _, sim = run1(net, ext_from_ticks(8, 1, 1, [(0, 0, 0)]), 8, lib)
    assert _events_str(ev) == g["two_hop"]["out"], _events_str(ev)
    assert cnt["hops"] == int(g["two_hop"]["hops"])
    assert np.array_equal(sim.links(), _links_of(g["two_hop"]["links"], 4)), sim.links().tolist()


def _links_of(text, C):
    out = np.zeros((C, 4), np.int64)
    for item in text.split(";"):
        c, d, k = (int(x) for x in item.split())
        out[c, d] = k
    return out


def pin_link_counts(lib=None):
    """Packets per mesh link on the XY route (Sec. III-D, Fig. 2: packets hop
    through the routers of the cores between source and destination)."""
    g = parse_golden("routing_cases.txt")["ping_pong"]
    dk = np.zeros((12, 1), np.uint8)
    dx = np.zeros((12, 1), np.int16)
    dy = np.zeros((12, 1), np.int16)
    dd = np.zeros((12, 1), np.uint8)
    dk[0], dx[0], dy[0], dd[0] = W.DEST_CORE, 3, 2, 1
    dk[11], dx[11], dy[11], dd[11] = W.DEST_CORE, -3, -2, 1
    net = make_net(12, 1, 1, G=1, grid_w=4, weight=10, threshold=10, dest_kind=dk, dest_dx=dx, dest_dy=dy,
                   dest_delay=dd, max_delay=1)
    _, _, cnt, st, _, sim = run1(net, ext_from_ticks(6, 1, 1, [(0, 0, 0)]), 6, lib, trace=True)
    assert [int(t) for t in np.nonzero(st[:, 0, 0])[0]] == [0, 2, 4]
    assert [int(t) for t in np.nonzero(st[:, 11, 0])[0]] == [1, 3, 5]
    assert cnt["hops"] == int(g["hops"])
    assert np.array_equal(sim.links(), _links_of(g["links"], 12)), sim.links().tolist()


def pin_or_merge(lib=None):
    g = parse_golden("routing_cases.txt")["or_merge"]
    conn = np.zeros((2, 1, 2), bool)
    conn[0, 0, :] = True
    conn[1, 0, 0] = True
    net = make_net(2, 1, 2, G=1, grid_w=2, conn=conn, weight=[[[10], [10]], [[5], [5]]],
                   threshold=[[10, 10], [6, 1000]],
                   dest_kind=[[W.DEST_CORE, W.DEST_CORE], [W.DEST_OUT, W.DEST_NONE]],
                   dest_dx=[[1, 1], [0, 0]], dest_delay=[[1, 1], [0, 0]], max_delay=2)
    ev, v, cnt, *_ = run1(net, ext_from_ticks(3, 1, 1, [(0, 0, 0)]), 3, lib)
    assert _events_str(ev) == g["out"], _events_str(ev)
    assert int(v[1, 0]) == int(g["v_core1_n0"]), int(v[1, 0])
    assert cnt["routed"] == int(g["routed"]) and cnt["delivered"] == int(g["delivered"]), cnt


def _tiny_random_net(r, seed):
    C = int(r.choice([1, 2, 3, 4]))
    gw = 2 if C == 4 and r.random() < 0.5 else C
    A, N = int(r.integers(1, 6)), int(r.integers(1, 6))
    G = int(r.integers(1, 5))
    b = int(r.integers(2, 10))
    P = int(r.choice([4, 6, 8, 32]))
    md = int(r.integers(1, 4))
    wmax = (1 << (b - 1)) - 1
    lim = (1 << (P - 1)) - 1
    net = W.random_net(seed, C, A, N, G, weight_bits=b, potential_bits=P, max_delay=md, grid_w=gw,
                       density=float(r.uniform(0.3, 1.0)), p_core=0.6, p_out=0.3,
                       leak_range=(-3, 3), thr_range=(1, max(2, min(lim, 2 * wmax))),
                       reset_range=(-2, 1), vinit_range=(-2, 2),
                       input_cores=sorted(set(r.integers(0, C, size=int(r.integers(1, C + 1))).tolist())),
                       config_id=500,
                       floor_range=(-6, 0) if r.random() < 0.3 else None,
                       linear_frac=float(r.choice([0.0, 0.0, 0.5, 1.0])))
    return net


def _compare_with_brute(net, ext, T, lib):
    ev, v, cnt, st, vt, sim = run1(net, ext, T, lib, trace=True)
    bev, bV, bcnt, _, per_tick = brute_simulate(net, ext, T)
    assert np.array_equal(sim.links(), np.array(bcnt["links"], np.int64).reshape(-1, 4)), "link counts differ"
    assert cnt["hops"] == sum(bcnt["links"])
    assert [tuple(int(x) for x in e) for e in ev] == bev, "output spikes differ"
    assert np.array_equal(v, np.array(bV, dtype=np.int64).astype(np.int32)), "potentials differ"
    for k in ("emitted", "routed", "delivered", "out", "events"):
        assert cnt[k] == bcnt[k], (k, cnt[k], bcnt[k])
    for t in range(T):
        got = {(int(c), int(n)) for c, n in zip(*np.nonzero(st[t]))}
        assert got == set(per_tick[t]), f"spike set differs at tick {t}"


def pin_brute_force_random(lib=None, n=150, seed=3):
    r = np.random.default_rng(seed)
    for i in range(n):
        net = _tiny_random_net(r, 10_000 + i)
        T = int(r.integers(1, 9))
        ext = (r.random((T, len(net.input_cores), net.num_axons)) < r.uniform(0.2, 0.9))
        ext = W.pack_bits(ext)
        _compare_with_brute(net, ext, T, lib)


def pin_brute_force_exhaustive(lib=None, n_params=3, seed=4):
    """All 2^(A*T) input patterns (A=3 axons, T=4 ticks) on a 2-core net."""
    r = np.random.default_rng(seed)
    A, T = 3, 4
    for p in range(n_params):
        net = W.random_net(20_000 + p, 2, A, 3, 2, weight_bits=4, potential_bits=6, max_delay=2,
                           density=0.7, p_core=0.7, p_out=0.3, leak_range=(-1, 1),
                           thr_range=(1, 9), reset_range=(-1, 0), input_cores=[0], config_id=501)
        pats = np.arange(1 << (A * T))
        bits = ((pats[:, None] >> np.arange(A * T)[None, :]) & 1).astype(bool).reshape(-1, T, 1, A)
        exts = W.pack_bits(bits)                       # [P, T, 1, 1]
        res = O.simulate(net, exts, T, lib=lib)
        for i in range(0, len(pats), max(1, len(pats) // 512)):
            bev, bV, bcnt, *_ = brute_simulate(net, exts[i], T)
            assert [tuple(int(x) for x in e) for e in res[i]["events"]] == bev, (p, i)
            assert np.array_equal(res[i]["v"], np.array(bV, dtype=np.int32)), (p, i)
            assert res[i]["counters"]["delivered"] == bcnt["delivered"], (p, i)


def pin_invariants(lib=None, seed=5):
    net = W.random_net(30_000, 6, 64, 96, 4, weight_bits=9, potential_bits=12, max_delay=5,
                       grid_w=3, density=0.3, p_core=0.6, p_out=0.3, leak_range=(-20, 20),
                       thr_range=(50, 400), reset_range=(-30, 10), vinit_range=(-100, 100),
                       input_cores=[0, 2, 5], config_id=502)
    T = 30
    ext = W.bernoulli_inputs(seed, net, 1, T, 0.3)[0]
    ev, v, cnt, st, vt, _ = run1(net, ext, T, lib, trace=True)
    kind = net.dest_kind
    emitted_core = int(sum((st[t].astype(bool) & (kind == W.DEST_CORE)).sum() for t in range(T)))
    emitted_out = int(sum((st[t].astype(bool) & (kind == W.DEST_OUT)).sum() for t in range(T)))
    assert cnt["routed"] == emitted_core
    assert cnt["out"] == emitted_out == len(ev)
    assert cnt["emitted"] == int(st.sum())
    assert cnt["delivered"] <= cnt["routed"]
    # every recorded output spike appears in the trace
    for t, c, n in ev:
        assert st[t, c, n] == 1 and kind[c, n] == W.DEST_OUT
    # potential bounds: either the reset value right after a spike or inside
    # [-2^(P-1), threshold - 1]
    lo = -(1 << (net.potential_bits - 1))
    for t in range(T):
        fired = st[t].astype(bool)
        assert np.all(vt[t][fired] == net.reset[fired])
        nf = ~fired
        assert np.all(vt[t][nf] >= lo) and np.all(vt[t][nf] <= net.threshold[nf] - 1)
    assert cnt["hops"] == int(sum(
        (st[t].astype(bool) & (kind == W.DEST_CORE)).astype(np.int64).ravel()
        @ (np.abs(net.dest_dx.astype(np.int64)) + np.abs(net.dest_dy.astype(np.int64))).ravel()
        for t in range(T)))
    links = O.OracleSim(net, lib)
    links.run(ext, T)
    assert int(links.links().sum()) == cnt["hops"]
    # every hop leaves a core towards a neighbour inside the mesh
    lk = links.links().reshape(net.grid_h, net.grid_w, 4)
    assert not lk[:, -1, 0].any() and not lk[:, 0, 1].any() and not lk[-1, :, 2].any() and not lk[0, :, 3].any()
    # silence without drive: no input, leak <= 0, V0 <= 0, threshold > 0
    quiet = W.random_net(30_001, 4, 32, 32, 2, leak_range=(-5, 0), thr_range=(1, 100),
                         vinit_range=(-50, 0), config_id=503)
    ev2, _, cnt2, *_ = run1(quiet, None, 20, lib)
    assert len(ev2) == 0 and cnt2["emitted"] == 0


def pin_resume_and_prefix(lib=None, seed=6):
    net = W.random_net(40_000, 4, 64, 64, 4, max_delay=6, grid_w=2, density=0.3, p_core=0.7,
                       p_out=0.3, input_cores=[0, 1], config_id=504)
    T1, T2 = 7, 11
    ext = W.bernoulli_inputs(seed, net, 1, T1 + T2, 0.25)[0]
    ev, v, cnt, *_ = run1(net, ext, T1 + T2, lib)
    sim = O.OracleSim(net, lib)
    e1, *_ = sim.run(ext[:T1], T1)
    e2, *_ = sim.run(ext[T1:], T2)
    assert np.array_equal(np.concatenate([e1, e2]), ev)
    assert np.array_equal(sim.potentials(), v)
    assert sim.counters() == cnt
    ep, *_ = run1(net, ext, T1, lib)
    assert np.array_equal(ep, ev[ev[:, 0] < T1])


def pin_relabel(lib=None, seed=7):
    """Relabeling cores on a 1-row mesh permutes the results."""
    C = 6
    net = W.random_net(50_000, C, 32, 48, 3, max_delay=3, density=0.35, p_core=0.7, p_out=0.3,
                       input_cores=[1, 4], config_id=505)
    T = 12
    ext = W.bernoulli_inputs(seed, net, 1, T, 0.4)[0]
    ev, v, *_ = run1(net, ext, T, lib)
    perm = np.random.default_rng(seed).permutation(C)        # old core c -> new label perm[c]
    inv = np.argsort(perm)
    src_new = np.repeat(np.arange(C)[:, None], net.num_neurons, axis=1)
    dest_old = (np.arange(C)[:, None] + net.dest_dx.astype(np.int64))     # 1-row mesh: dest = c + dx
    dest_new = perm[dest_old[inv]]
    dx = np.where(net.dest_kind[inv] == W.DEST_CORE, dest_new - src_new, 0)
    net2 = W.Net(C, net.num_axons, net.num_neurons, net.num_types, net.weight_bits,
                 net.potential_bits, net.max_delay, C, 1, net.crossbar[inv], net.axon_type[inv],
                 net.weight[inv], net.leak[inv], net.threshold[inv], net.reset[inv],
                 net.v_init[inv], net.dest_kind[inv], dx.astype(np.int16), net.dest_dy[inv],
                 net.dest_axon[inv], net.dest_delay[inv],
                 np.asarray([perm[c] for c in net.input_cores], np.int32)).contiguous()
    ev2, v2, *_ = run1(net2, ext, T, lib)
    assert np.array_equal(v2, v[inv])
    mapped = sorted((int(t), int(perm[c]), int(n)) for t, c, n in ev)
    assert [tuple(int(x) for x in e) for e in ev2] == mapped


ALL_PINS = [pin_single_neuron_cases, pin_neuron_model_cases, pin_linear_reset_sweep, pin_floor_sweep,
            pin_value_widths, pin_closed_form_sweep, pin_axon_types,
            pin_integration_matmul, pin_delay_delivery, pin_link_counts, pin_or_merge,
            pin_brute_force_random, pin_brute_force_exhaustive, pin_invariants,
            pin_resume_and_prefix, pin_relabel]
