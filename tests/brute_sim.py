"""Independent pure-Python RANC simulator for tiny networks (test pin for the oracle).

It shares no code with the oracle or the HIP path and uses different data
structures on purpose: deliveries are kept as a dictionary from absolute tick
to a set of (core, axon) pairs instead of a per-core ring of scheduler rows,
destinations are computed in one step from the relative mesh offset (the
direct routing of GPU-RANC Sec. III-D) instead of hop by hop, and the
integration is a Python sum over the axons of each neuron.

Semantics (GPU-RANC Sec. II and Algorithm 1, with the readings the oracle
uses): an axon holds a spike at tick t if any packet for (core, axon, t) was
sent or the external input has it; a neuron's input is the sum, over spiking
connected axons, of its weight for the axon's type; U = V + input + leak is
clamped to a signed potential_bits range; the neuron fires iff U >= threshold
and is then set to its reset value (or, in linear-reset mode, to U minus the
threshold, clamped to the range); a neuron that does not fire keeps
max(U, floor) when it has a floor; a spike at t with delay d reaches its
destination axon at t + d. Only for tiny cases: it is slow on purpose.
"""
from __future__ import annotations

from collections import defaultdict


def _bit(words, i):
    return (int(words[i >> 5]) >> (i & 31)) & 1


def brute_simulate(net, ext, T, pending=None, V=None, t0=0):
    """Simulate one instance for ticks t0 .. t0+T-1.

    ``ext`` is indexable as ext[t - t0][k][word] (or None). Returns
    (events list of (tick, core, neuron), V list-of-lists, counters dict,
    pending dict, per-tick spike lists).
    """
    Cn, A, N = net.num_cores, net.num_axons, net.num_neurons
    gw = net.grid_w
    lo = -(1 << (net.potential_bits - 1))
    hi = (1 << (net.potential_bits - 1)) - 1
    if V is None:
        V = [[int(net.v_init[c][n]) for n in range(N)] for c in range(Cn)]
    if pending is None:
        pending = defaultdict(set)
    counters = dict(emitted=0, routed=0, delivered=0, out=0, events=0, links=[0] * (4 * Cn))
    events = []
    per_tick = []
    for t in range(t0, t0 + T):
        arrived = pending.pop(t, set())
        counters["delivered"] += len(arrived)
        active = set(arrived)
        if ext is not None:
            for k, c in enumerate(net.input_cores):
                for a in range(A):
                    if _bit(ext[t - t0][k], a):
                        active.add((int(c), a))
        fired = []
        for c in range(Cn):
            for n in range(N):
                total = 0
                for a in range(A):
                    if (c, a) in active and _bit(net.crossbar[c][a], n):
                        total += int(net.weight[c][n][int(net.axon_type[c][a])])
                        counters["events"] += 1
                u = V[c][n] + total + int(net.leak[c][n])
                u = min(hi, max(lo, u))
                theta = int(net.threshold[c][n])
                if u >= theta:
                    linear = net.reset_mode is not None and int(net.reset_mode[c][n]) == 1
                    V[c][n] = min(hi, max(lo, u - theta)) if linear else int(net.reset[c][n])
                    fired.append((c, n))
                elif net.floor is not None:
                    V[c][n] = max(u, int(net.floor[c][n]))
                else:
                    V[c][n] = u
        counters["emitted"] += len(fired)
        for (c, n) in fired:
            kind = int(net.dest_kind[c][n])
            if kind == 2:
                events.append((t, c, n))
                counters["out"] += 1
            elif kind == 1:
                x = c % gw + int(net.dest_dx[c][n])
                y = c // gw + int(net.dest_dy[c][n])
                assert 0 <= x < gw and 0 <= y < net.grid_h
                # the links of the x-then-y route: x from the source column to
                # the destination column on the source row, then y along the
                # destination column; each hop counted at the core it leaves
                sx, sy = c % gw, c // gw
                for xi in (range(sx, x) if x > sx else range(sx, x, -1)):
                    counters["links"][4 * (sy * gw + xi) + (0 if x > sx else 1)] += 1
                for yi in (range(sy, y) if y > sy else range(sy, y, -1)):
                    counters["links"][4 * (yi * gw + x) + (2 if y > sy else 3)] += 1
                pending[t + int(net.dest_delay[c][n])].add((y * gw + x, int(net.dest_axon[c][n])))
                counters["routed"] += 1
        per_tick.append(fired)
    return events, V, counters, pending, per_tick
