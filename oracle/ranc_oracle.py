"""ctypes wrapper around the serial RANC oracle (``ranc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the benchmark's CPU-baseline leg. The simulation package never imports it.

Samples are independent network instances, so :func:`simulate` runs them on a
thread pool (the C code releases the GIL through ctypes); each instance is
simulated serially tick by tick as in GPU-RANC Algorithm 1.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading
from concurrent.futures import ThreadPoolExecutor

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ranc_oracle.c")
_LIB = os.path.join(_HERE, "libranc_oracle.so")

ORC_OK, ORC_TRUNCATED = 0, 1
COUNTER_NAMES = ("emitted", "routed", "delivered", "out", "events", "hops")


def build(force: bool = True) -> str:
    """Compile the oracle with plain gcc (portable flags, no -march=native)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-Wall", "-Wextra", "-fPIC", "-shared",
                               _SRC, "-o", tmp])
        os.replace(tmp, _LIB)
    return _LIB


class _Net(C.Structure):
    _fields_ = [(n, C.c_int32) for n in ("num_cores", "num_axons", "num_neurons", "num_types",
                                          "weight_bits", "potential_bits", "max_delay",
                                          "grid_w", "grid_h")] + [
        ("crossbar", C.c_void_p), ("axon_type", C.c_void_p), ("weight", C.c_void_p),
        ("leak", C.c_void_p), ("threshold", C.c_void_p), ("reset", C.c_void_p),
        ("v_init", C.c_void_p), ("dest_kind", C.c_void_p), ("dest_dx", C.c_void_p),
        ("dest_dy", C.c_void_p), ("dest_axon", C.c_void_p), ("dest_delay", C.c_void_p),
        ("num_input_cores", C.c_int32), ("input_cores", C.c_void_p),
        ("leak_bits", C.c_int32), ("reset_bits", C.c_int32), ("floor", C.c_void_p), ("reset_mode", C.c_void_p)]


def _bind(path: str):
    lib = C.CDLL(path)
    lib.orc_new.restype = C.c_void_p
    lib.orc_new.argtypes = [C.POINTER(_Net)]
    lib.orc_check.restype = C.c_int
    lib.orc_check.argtypes = [C.POINTER(_Net)]
    lib.orc_free.argtypes = [C.c_void_p]
    lib.orc_run.restype = C.c_int
    lib.orc_run.argtypes = [C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p, C.c_int64,
                            C.POINTER(C.c_int64), C.c_void_p, C.c_void_p]
    lib.orc_potentials.argtypes = [C.c_void_p, C.c_void_p]
    lib.orc_counters.argtypes = [C.c_void_p, C.c_void_p]
    lib.orc_links.argtypes = [C.c_void_p, C.c_void_p]
    lib.orc_tick.restype = C.c_int64
    lib.orc_tick.argtypes = [C.c_void_p]
    return lib


_lib = None
_lib_lock = threading.Lock()


def _load():
    global _lib
    with _lib_lock:
        if _lib is None:
            if not os.path.exists(_LIB):
                build(force=False)
            _lib = _bind(_LIB)
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


class _NetHolder:
    """Keeps the numpy arrays alive and exposes the C struct."""

    def __init__(self, net):
        self.arrays = dict(
            crossbar=np.ascontiguousarray(net.crossbar, dtype=np.uint32),
            axon_type=np.ascontiguousarray(net.axon_type, dtype=np.uint8),
            weight=np.ascontiguousarray(net.weight, dtype=np.int16),
            leak=np.ascontiguousarray(net.leak, dtype=np.int32),
            threshold=np.ascontiguousarray(net.threshold, dtype=np.int32),
            reset=np.ascontiguousarray(net.reset, dtype=np.int32),
            v_init=np.ascontiguousarray(net.v_init, dtype=np.int32),
            dest_kind=np.ascontiguousarray(net.dest_kind, dtype=np.uint8),
            dest_dx=np.ascontiguousarray(net.dest_dx, dtype=np.int16),
            dest_dy=np.ascontiguousarray(net.dest_dy, dtype=np.int16),
            dest_axon=np.ascontiguousarray(net.dest_axon, dtype=np.uint16),
            dest_delay=np.ascontiguousarray(net.dest_delay, dtype=np.uint8),
            input_cores=np.ascontiguousarray(net.input_cores, dtype=np.int32),
        )
        floor = getattr(net, "floor", None)
        mode = getattr(net, "reset_mode", None)
        if floor is not None:
            self.arrays["floor"] = np.ascontiguousarray(floor, dtype=np.int32)
        if mode is not None:
            self.arrays["reset_mode"] = np.ascontiguousarray(mode, dtype=np.uint8)
        self.c = _Net(net.num_cores, net.num_axons, net.num_neurons, net.num_types,
                      net.weight_bits, net.potential_bits, net.max_delay, net.grid_w, net.grid_h,
                      *[_ptr(self.arrays[k]) for k in ("crossbar", "axon_type", "weight", "leak",
                                                      "threshold", "reset", "v_init", "dest_kind",
                                                      "dest_dx", "dest_dy", "dest_axon",
                                                      "dest_delay")],
                      len(self.arrays["input_cores"]), _ptr(self.arrays["input_cores"]),
                      int(getattr(net, "leak_bits", 32)), int(getattr(net, "reset_bits", 32)),
                      _ptr(self.arrays["floor"]) if floor is not None else None,
                      _ptr(self.arrays["reset_mode"]) if mode is not None else None)
        self.C, self.N = net.num_cores, net.num_neurons


def check(net, lib=None) -> int:
    h = _NetHolder(net)
    return (lib if lib is not None else _load()).orc_check(C.byref(h.c))


def build_variant(src_text: str, out_path: str, extra_flags=(), bind: bool = True):
    """Compile an alternative oracle source (used to check that the pins catch
    deliberate mistakes planted in a copy of the oracle, or to build the oracle
    with the address and undefined-behaviour sanitizers) and bind it."""
    src = out_path + ".c"
    with open(src, "w") as f:
        f.write(src_text)
    subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", *extra_flags, src, "-o", out_path])
    return _bind(out_path) if bind else out_path


def source_text() -> str:
    with open(_SRC) as f:
        return f.read()


class OracleSim:
    """One independent network instance, resumable across :meth:`run` calls."""

    def __init__(self, net, lib=None):
        self._h = _NetHolder(net)
        self._lib = lib if lib is not None else _load()
        self._p = self._lib.orc_new(C.byref(self._h.c))
        if not self._p:
            raise ValueError(f"oracle rejected the network (orc_check={check(net)})")

    def __del__(self):
        p, self._p = getattr(self, "_p", None), None
        if p:
            self._lib.orc_free(p)

    @property
    def tick(self) -> int:
        return int(self._lib.orc_tick(self._p))

    def run(self, ext: np.ndarray | None, T: int, trace: bool = False, cap: int | None = None):
        """Run T ticks. ``ext`` is [T, C_in, ceil(A/32)] uint32 or None.

        Returns (events int64 [n, 3] of (tick, core, neuron), spike_trace, v_trace).
        """
        Cc, N = self._h.C, self._h.N
        if ext is not None:
            ext = np.ascontiguousarray(ext, dtype=np.uint32)
            assert ext.shape[0] >= T
        if cap is None:
            cap = T * Cc * N
        ev = np.empty((max(cap, 1), 3), dtype=np.int64)
        n_out = C.c_int64(0)
        st = np.empty((T, Cc, N), dtype=np.uint8) if trace else None
        vt = np.empty((T, Cc, N), dtype=np.int32) if trace else None
        rc = self._lib.orc_run(self._p, _ptr(ext) if ext is not None else None, T, _ptr(ev), cap,
                               C.byref(n_out), _ptr(st) if trace else None,
                               _ptr(vt) if trace else None)
        if rc < 0:
            raise RuntimeError(f"oracle run failed: {rc}")
        if rc == ORC_TRUNCATED:
            raise RuntimeError("oracle event buffer too small")
        return ev[: n_out.value].copy(), st, vt

    def potentials(self) -> np.ndarray:
        out = np.empty((self._h.C, self._h.N), dtype=np.int32)
        self._lib.orc_potentials(self._p, _ptr(out))
        return out

    def links(self) -> np.ndarray:
        """Packets per mesh link since the start, int64 [C, 4]: out of core c
        towards +x, -x, +y, -y."""
        out = np.zeros((self._h.C, 4), dtype=np.int64)
        self._lib.orc_links(self._p, _ptr(out))
        return out

    def counters(self) -> dict:
        out = np.zeros(len(COUNTER_NAMES), dtype=np.int64)
        self._lib.orc_counters(self._p, _ptr(out))
        return dict(zip(COUNTER_NAMES, (int(x) for x in out)))


def default_threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(n, 16))


def simulate(net, inputs: np.ndarray | None, T: int, samples=None, threads: int | None = None,
             trace: bool = False, lib=None):
    """Simulate independent samples from V = v_init and an empty scheduler.

    ``inputs`` is [S, T, C_in, ceil(A/32)] (or None). ``samples`` selects which
    sample indices to run (default: all). Returns a list of dicts with keys
    ``events`` (int64 [n,3]), ``v`` (int32 [C,N]), ``counters`` and, if
    ``trace``, ``spikes`` [T,C,N] and ``vtrace`` [T,C,N].
    """
    if samples is None:
        samples = range(inputs.shape[0] if inputs is not None else 1)
    samples = list(samples)

    def one(s):
        sim = OracleSim(net, lib)
        ext = inputs[s, :T] if inputs is not None else None
        ev, st, vt = sim.run(ext, T, trace=trace)
        r = dict(sample=s, events=ev, v=sim.potentials(), counters=sim.counters(), links=sim.links())
        if trace:
            r["spikes"], r["vtrace"] = st, vt
        return r

    threads = threads or default_threads()
    if threads == 1 or len(samples) == 1:
        return [one(s) for s in samples]
    with ThreadPoolExecutor(max_workers=threads) as ex:
        return list(ex.map(one, samples))
