"""Thin ctypes binding of the C ABI in ``include/ranc.h``.

The functions below carry the C names and only marshal arguments; every step
of the simulation runs in the HIP library ``libranc.so``. PyTorch supplies the
device memory (the workspace is a ``torch.uint8`` CUDA tensor owned by the
caller) and the stream (``torch.cuda.current_stream()``). If the library is
not built, importing the binding raises: there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libranc.so")

RANC_ABI_VERSION = 2
RANC_OK, RANC_EINVAL, RANC_ERANGE, RANC_ENOMEM, RANC_EDEVICE, RANC_ESTATE, RANC_ETRUNC, RANC_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5, -6, -7
RANC_ETIMEOUT = -8
STATUS_NAMES = {0: "RANC_OK", -1: "RANC_EINVAL", -2: "RANC_ERANGE", -3: "RANC_ENOMEM", -4: "RANC_EDEVICE",
                -5: "RANC_ESTATE", -6: "RANC_ETRUNC", -7: "RANC_EUNSUPPORTED", -8: "RANC_ETIMEOUT"}
RANC_PATH_AUTO, RANC_PATH_PLAIN, RANC_PATH_MFMA, RANC_PATH_SPARSE = 0, 1, 2, 3
PATHS = {"auto": RANC_PATH_AUTO, "plain": RANC_PATH_PLAIN, "mfma": RANC_PATH_MFMA, "sparse": RANC_PATH_SPARSE}
RANC_RESET_ABSOLUTE, RANC_RESET_LINEAR = 0, 1
RANC_INPUTS_ON_DEVICE = 1
RANC_RUN_GRAPH = 2
RANC_BATCH_PERSISTENT = 4
RANC_RUN_RESIDENT = 8

EXPORTED = ("ranc_last_error", "ranc_workspace_bytes", "ranc_load_network", "ranc_run_ticks",
            "ranc_read_spikes", "ranc_read_potentials", "ranc_read_counters", "ranc_current_tick",
            "ranc_get_path", "ranc_profile_enable", "ranc_profile_read", "ranc_reset_state", "ranc_free",
            "ranc_autotune", "ranc_set_launch_shape", "ranc_get_launch_shape", "ranc_load_network_static",
            "ranc_link_counts_enable", "ranc_read_links", "ranc_raster_bytes", "ranc_copy_raster",
            "ranc_output_neurons")
RANC_LINK_XPLUS, RANC_LINK_XMINUS, RANC_LINK_YPLUS, RANC_LINK_YMINUS = 0, 1, 2, 3
RANC_RASTER_BY_NEURON, RANC_RASTER_BY_SAMPLE = 0, 1
RASTER_LAYOUTS = {"neuron": RANC_RASTER_BY_NEURON, "sample": RANC_RASTER_BY_SAMPLE}
RANC_STATIC_WORKSPACE_BYTES = 64 << 20


class RancError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class ranc_net_desc(C.Structure):
    _fields_ = [("abi_version", C.c_uint32)] + [
        (n, C.c_int32) for n in ("num_cores", "num_axons", "num_neurons", "num_types", "weight_bits",
                                 "potential_bits", "max_delay", "grid_w", "grid_h")] + [
        ("crossbar", C.c_void_p), ("axon_type", C.c_void_p), ("weight", C.c_void_p), ("leak", C.c_void_p),
        ("threshold", C.c_void_p), ("reset", C.c_void_p), ("v_init", C.c_void_p), ("dest_kind", C.c_void_p),
        ("dest_dx", C.c_void_p), ("dest_dy", C.c_void_p), ("dest_axon", C.c_void_p), ("dest_delay", C.c_void_p),
        ("num_input_cores", C.c_int32), ("input_cores", C.c_void_p),
        ("leak_bits", C.c_int32), ("reset_bits", C.c_int32), ("floor", C.c_void_p), ("reset_mode", C.c_void_p)]


class ranc_spike(C.Structure):
    _fields_ = [("tick", C.c_int64), ("core", C.c_int32), ("neuron", C.c_int32)]


class ranc_profile(C.Structure):
    _fields_ = [("integrate_ms", C.c_double), ("route_ms", C.c_double),
                ("integrate_launches", C.c_int64), ("route_launches", C.c_int64),
                ("graph_ms", C.c_double), ("graph_launches", C.c_int64),
                ("graphs_held", C.c_int64), ("graphs_dropped", C.c_int64),
                ("resident_ms", C.c_double), ("resident_launches", C.c_int64)]


class ranc_counters(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in ("emitted", "routed", "delivered", "out", "events")]


class ranc_tune(C.Structure):
    _fields_ = [("samples_per_wg", C.c_int32), ("route_samples_per_block", C.c_int32),
                ("route_split", C.c_int32), ("route_stage", C.c_int32),
                ("ms_per_tick", C.c_double), ("candidates", C.c_int32), ("route_lanes_per_word", C.c_int32)]


SPIKE_DTYPE = np.dtype([("tick", "<i8"), ("core", "<i4"), ("neuron", "<i4")])


def _load_lib():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build() "
                          "(python paper_2404_16208_amd/build.py)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, i64, u32, sz = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_size_t
    sig = {
        "ranc_last_error": (C.c_char_p, []),
        "ranc_workspace_bytes": (C.c_int, [C.POINTER(ranc_net_desc), i32, i32, i32, C.POINTER(sz)]),
        "ranc_load_network": (C.c_int, [C.POINTER(ranc_net_desc), i32, i32, i32, vp, sz, vp, C.POINTER(vp)]),
        "ranc_load_network_static": (C.c_int, [C.POINTER(ranc_net_desc), i32, i32, i32, vp, C.POINTER(vp)]),
        "ranc_run_ticks": (C.c_int, [C.POINTER(vp), i32, C.POINTER(vp), u32, i32, vp]),
        "ranc_read_spikes": (C.c_int, [vp, i32, i64, i64, vp, i64, C.POINTER(i64)]),
        "ranc_read_potentials": (C.c_int, [vp, i32, vp]),
        "ranc_read_counters": (C.c_int, [vp, i32, C.POINTER(ranc_counters)]),
        "ranc_current_tick": (C.c_int, [vp, C.POINTER(i64)]),
        "ranc_link_counts_enable": (C.c_int, [vp, i32]),
        "ranc_raster_bytes": (C.c_int, [vp, i64, u32, C.POINTER(sz)]),
        "ranc_copy_raster": (C.c_int, [vp, i64, i64, u32, vp, sz, vp]),
        "ranc_output_neurons": (C.c_int, [vp, vp, i64, C.POINTER(i64)]),
        "ranc_read_links": (C.c_int, [vp, i32, vp]),
        "ranc_get_path": (C.c_int, [vp, C.POINTER(i32)]),
        "ranc_profile_enable": (C.c_int, [vp, i32]),
        "ranc_profile_read": (C.c_int, [vp, C.POINTER(ranc_profile)]),
        "ranc_reset_state": (C.c_int, [vp, vp]),
        "ranc_free": (None, [vp]),
        "ranc_autotune": (C.c_int, [vp, vp, u32, i32, vp, C.POINTER(ranc_tune)]),
        "ranc_set_launch_shape": (C.c_int, [vp, C.POINTER(ranc_tune)]),
        "ranc_get_launch_shape": (C.c_int, [vp, C.POINTER(ranc_tune)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    return lib


_lib = _load_lib()


def _check(status):
    if status != RANC_OK:
        raise RancError(status, ranc_last_error())
    return status


# ------------------------------------------------------------- C names

def ranc_last_error() -> str:
    return _lib.ranc_last_error().decode()


class Desc:
    """A ranc_net_desc plus the contiguous numpy arrays it points to."""

    def __init__(self, net):
        a = lambda x, dt: np.ascontiguousarray(x, dtype=dt)
        self.arrays = dict(crossbar=a(net.crossbar, np.uint32), axon_type=a(net.axon_type, np.uint8),
                           weight=a(net.weight, np.int16), leak=a(net.leak, np.int32),
                           threshold=a(net.threshold, np.int32), reset=a(net.reset, np.int32),
                           v_init=a(net.v_init, np.int32), dest_kind=a(net.dest_kind, np.uint8),
                           dest_dx=a(net.dest_dx, np.int16), dest_dy=a(net.dest_dy, np.int16),
                           dest_axon=a(net.dest_axon, np.uint16), dest_delay=a(net.dest_delay, np.uint8),
                           input_cores=a(net.input_cores, np.int32))
        floor, mode = getattr(net, "floor", None), getattr(net, "reset_mode", None)
        if floor is not None:
            self.arrays["floor"] = a(floor, np.int32)
        if mode is not None:
            self.arrays["reset_mode"] = a(mode, np.uint8)
        p = {k: v.ctypes.data for k, v in self.arrays.items()}
        self.c = ranc_net_desc(RANC_ABI_VERSION, net.num_cores, net.num_axons, net.num_neurons, net.num_types,
                               net.weight_bits, net.potential_bits, net.max_delay, net.grid_w, net.grid_h,
                               p["crossbar"], p["axon_type"], p["weight"], p["leak"], p["threshold"], p["reset"],
                               p["v_init"], p["dest_kind"], p["dest_dx"], p["dest_dy"], p["dest_axon"],
                               p["dest_delay"], len(self.arrays["input_cores"]), p["input_cores"],
                               int(getattr(net, "leak_bits", 32)), int(getattr(net, "reset_bits", 32)),
                               p.get("floor"), p.get("reset_mode"))


def ranc_workspace_bytes(desc: Desc, num_samples: int, max_ticks_per_call: int, path: int = RANC_PATH_AUTO) -> int:
    out = C.c_size_t(0)
    _check(_lib.ranc_workspace_bytes(C.byref(desc.c), num_samples, max_ticks_per_call, path, C.byref(out)))
    return int(out.value)


def ranc_load_network(desc: Desc, num_samples: int, max_ticks_per_call: int, path: int, workspace_ptr: int,
                      workspace_bytes: int, stream: int) -> int:
    h = C.c_void_p(0)
    _check(_lib.ranc_load_network(C.byref(desc.c), num_samples, max_ticks_per_call, path, workspace_ptr,
                                  workspace_bytes, stream, C.byref(h)))
    return int(h.value)


def ranc_load_network_static(desc: Desc, num_samples: int, max_ticks_per_call: int, path: int, stream: int) -> int:
    h = C.c_void_p(0)
    _check(_lib.ranc_load_network_static(C.byref(desc.c), num_samples, max_ticks_per_call, path, stream,
                                         C.byref(h)))
    return int(h.value)


def ranc_run_ticks(handles, inputs_ptrs, flags: int, num_ticks: int, stream: int) -> None:
    n = len(handles)
    harr = (C.c_void_p * n)(*handles)
    iarr = (C.c_void_p * n)(*[p or None for p in inputs_ptrs]) if inputs_ptrs is not None else None
    _check(_lib.ranc_run_ticks(harr, n, iarr, flags, num_ticks, stream))


def ranc_read_spikes(handle: int, sample: int, tick_begin: int, tick_end: int, buf: np.ndarray | None = None):
    """Output-bus spikes of one sample in [tick_begin, tick_end). ``buf``: an
    optional SPIKE_DTYPE array to decode into (one call when it is large
    enough; a larger array is made otherwise). Returns (spikes, buffer): the
    spikes are a view of the buffer."""
    count = C.c_int64(0)
    if buf is None:
        buf = np.zeros(0, dtype=SPIKE_DTYPE)
    st = _lib.ranc_read_spikes(handle, sample, tick_begin, tick_end, buf.ctypes.data if len(buf) else None,
                               len(buf), C.byref(count))
    if st == RANC_ETRUNC:
        buf = np.zeros(max(int(count.value), 2 * len(buf)), dtype=SPIKE_DTYPE)
        st = _lib.ranc_read_spikes(handle, sample, tick_begin, tick_end, buf.ctypes.data, len(buf),
                                   C.byref(count))
    _check(st)
    return buf[:int(count.value)], buf


def ranc_read_potentials(handle: int, sample: int, C_: int, N: int) -> np.ndarray:
    out = np.empty((C_, N), dtype=np.int32)
    _check(_lib.ranc_read_potentials(handle, sample, out.ctypes.data))
    return out


def ranc_read_counters(handle: int, sample: int) -> dict:
    c = ranc_counters()
    _check(_lib.ranc_read_counters(handle, sample, C.byref(c)))
    return {k: int(getattr(c, k)) for k, _ in ranc_counters._fields_}


def ranc_link_counts_enable(handle: int, enable: bool) -> None:
    _check(_lib.ranc_link_counts_enable(handle, 1 if enable else 0))


def ranc_read_links(handle: int, sample: int, C_: int) -> np.ndarray:
    """Packets per mesh link of one sample, int64 [C, 4] (+x, -x, +y, -y)."""
    out = np.empty((C_, 4), dtype=np.int64)
    _check(_lib.ranc_read_links(handle, sample, out.ctypes.data))
    return out


def ranc_raster_bytes(handle: int, num_ticks: int, layout: int = RANC_RASTER_BY_SAMPLE) -> int:
    out = C.c_size_t(0)
    _check(_lib.ranc_raster_bytes(handle, num_ticks, layout, C.byref(out)))
    return int(out.value)


def ranc_copy_raster(handle: int, tick_begin: int, tick_end: int, layout: int, dst_ptr: int, dst_bytes: int,
                     stream: int) -> None:
    _check(_lib.ranc_copy_raster(handle, tick_begin, tick_end, layout, dst_ptr, dst_bytes, stream))


def ranc_output_neurons(handle: int) -> np.ndarray:
    """(core, neuron) of every output neuron, int32 [Nout, 2], in output-index order."""
    count = C.c_int64(0)
    st = _lib.ranc_output_neurons(handle, None, 0, C.byref(count))
    if st not in (RANC_OK, RANC_ETRUNC):
        _check(st)
    out = np.zeros((int(count.value), 2), dtype=np.int32)
    _check(_lib.ranc_output_neurons(handle, out.ctypes.data if len(out) else None, len(out), C.byref(count)))
    return out


def ranc_current_tick(handle: int) -> int:
    t = C.c_int64(0)
    _check(_lib.ranc_current_tick(handle, C.byref(t)))
    return int(t.value)


def ranc_get_path(handle: int) -> int:
    p = C.c_int32(0)
    _check(_lib.ranc_get_path(handle, C.byref(p)))
    return int(p.value)


def ranc_profile_enable(handle: int, enable: bool) -> None:
    _check(_lib.ranc_profile_enable(handle, 1 if enable else 0))


def ranc_profile_read(handle: int) -> dict:
    p = ranc_profile()
    _check(_lib.ranc_profile_read(handle, C.byref(p)))
    return {k: (float(getattr(p, k)) if k.endswith("_ms") else int(getattr(p, k))) for k, _ in ranc_profile._fields_}


def _tune_dict(t: ranc_tune) -> dict:
    return {k: (float(getattr(t, k)) if k == "ms_per_tick" else int(getattr(t, k))) for k, _ in ranc_tune._fields_}


def ranc_autotune(handle: int, inputs_ptr, flags: int, num_ticks: int, stream: int) -> dict:
    t = ranc_tune()
    _check(_lib.ranc_autotune(handle, inputs_ptr or None, flags, num_ticks, stream, C.byref(t)))
    return _tune_dict(t)


def ranc_set_launch_shape(handle: int, shape: dict) -> None:
    t = ranc_tune(**{k: shape.get(k, 0) for k, _ in ranc_tune._fields_})
    _check(_lib.ranc_set_launch_shape(handle, C.byref(t)))


def ranc_get_launch_shape(handle: int) -> dict:
    t = ranc_tune()
    _check(_lib.ranc_get_launch_shape(handle, C.byref(t)))
    return _tune_dict(t)


def ranc_reset_state(handle: int, stream: int) -> None:
    _check(_lib.ranc_reset_state(handle, stream))


def ranc_free(handle: int) -> None:
    _lib.ranc_free(handle)


# ------------------------------------------------------------- convenience

class RancNet:
    """A loaded network with its torch-owned workspace on the current CUDA device
    (or, with ``static_workspace``, in the library-held workspace of that
    device: ranc_load_network_static)."""

    def __init__(self, net, num_samples: int, max_ticks_per_call: int, path="auto", device="cuda",
                 static_workspace: bool = False, workspace_fill: int | None = None):
        import torch

        self.net = net
        self.S = num_samples
        self.RT = max_ticks_per_call
        self.desc = Desc(net)
        p = PATHS[path] if isinstance(path, str) else int(path)
        if static_workspace:
            self.workspace = None
            self.stream = torch.cuda.current_stream(torch.device(device))
            self.handle = ranc_load_network_static(self.desc, num_samples, max_ticks_per_call, p,
                                                   self.stream.cuda_stream)
        else:
            nbytes = ranc_workspace_bytes(self.desc, num_samples, max_ticks_per_call, p)
            self.workspace = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)
            if workspace_fill is not None:   # e.g. a poison byte, to show nothing reads unwritten memory
                self.workspace.fill_(workspace_fill)
            self.stream = torch.cuda.current_stream(self.workspace.device)
            self.handle = ranc_load_network(self.desc, num_samples, max_ticks_per_call, p,
                                            self.workspace.data_ptr(), self.workspace.numel(),
                                            self.stream.cuda_stream)
        self.path = {RANC_PATH_PLAIN: "plain", RANC_PATH_MFMA: "mfma", RANC_PATH_SPARSE: "sparse"}[ranc_get_path(self.handle)]

    def close(self):
        if getattr(self, "handle", None):
            ranc_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def tick(self) -> int:
        return ranc_current_tick(self.handle)

    def run(self, inputs, num_ticks: int, graph: bool = False, resident: bool = False):
        """Advance by num_ticks. ``inputs``: None, a numpy uint32 array or a CUDA tensor
        (int32/uint32 bits) of shape [S, num_ticks, C_in, A/32]. ``graph``: run the
        ticks as one captured HIP graph (captured on first use, then replayed).
        ``resident``: run them in one state-resident persistent launch
        (RANC_RUN_RESIDENT; synchronizes the stream)."""
        flags = (RANC_RUN_GRAPH if graph else 0) | (RANC_RUN_RESIDENT if resident else 0)
        ptr, keep = None, None
        if inputs is not None:
            if isinstance(inputs, np.ndarray):
                keep = np.ascontiguousarray(inputs, dtype=np.uint32)
                assert keep.shape[:2] == (self.S, num_ticks), keep.shape
                ptr = keep.ctypes.data
            else:
                assert inputs.is_cuda and inputs.is_contiguous() and inputs.element_size() == 4
                assert tuple(inputs.shape[:2]) == (self.S, num_ticks), tuple(inputs.shape)
                flags, ptr, keep = flags | RANC_INPUTS_ON_DEVICE, inputs.data_ptr(), inputs
        ranc_run_ticks([self.handle], [ptr] if ptr else None, flags, num_ticks, self.stream.cuda_stream)
        if isinstance(keep, np.ndarray):
            self.stream.synchronize()   # host buffer must outlive the staging copy
        return self

    def spikes(self, sample: int, tick_begin: int | None = None, tick_end: int | None = None) -> np.ndarray:
        t = self.tick
        if tick_end is None:
            tick_end = t
        if tick_begin is None:
            tick_begin = max(0, t - self.RT)
        sp, self._spike_buf = ranc_read_spikes(self.handle, sample, tick_begin, tick_end,
                                               getattr(self, "_spike_buf", None))
        return np.stack([sp["tick"], sp["core"].astype(np.int64), sp["neuron"].astype(np.int64)], axis=1) \
            if len(sp) else np.zeros((0, 3), np.int64)

    def raster_bytes(self, num_ticks: int, layout: str = "sample") -> int:
        return ranc_raster_bytes(self.handle, num_ticks, RASTER_LAYOUTS[layout])

    def copy_raster(self, tick_begin: int, tick_end: int, dst, layout: str = "sample", stream=None):
        """Queue the bulk copy of ticks [tick_begin, tick_end) of every sample's
        output-bus spikes into ``dst`` (a CUDA tensor, or a pinned host tensor, of
        at least raster_bytes(T, layout) bytes). layout "sample": u32 words
        [T][S][ceil(Nout/32)], bit o % 32 of word (t, s, o // 32); "neuron": u64
        words [T][Nout][ceil(S/64)], bit i of word (t, o, w) = sample 64 w + i.
        ``stream``: a torch stream (default: the handle's stream)."""
        st = (stream or self.stream).cuda_stream
        ranc_copy_raster(self.handle, tick_begin, tick_end, RASTER_LAYOUTS[layout], dst.data_ptr(),
                         dst.numel() * dst.element_size(), st)
        return dst

    def output_neurons(self) -> np.ndarray:
        if getattr(self, "_out_neurons", None) is None:
            self._out_neurons = ranc_output_neurons(self.handle)
        return self._out_neurons

    def potentials(self, sample: int) -> np.ndarray:
        return ranc_read_potentials(self.handle, sample, self.net.num_cores, self.net.num_neurons)

    def counters(self, sample: int) -> dict:
        return ranc_read_counters(self.handle, sample)

    def count_links(self, enable: bool = True):
        """Count packets per mesh link on the ticks run from now on."""
        ranc_link_counts_enable(self.handle, enable)
        return self

    def links(self, sample: int) -> np.ndarray:
        """Packets per mesh link of one sample since load or reset, int64 [C, 4]:
        out of core c towards +x, -x, +y, -y."""
        return ranc_read_links(self.handle, sample, self.net.num_cores)

    def reset(self):
        ranc_reset_state(self.handle, self.stream.cuda_stream)
        return self

    def autotune(self, inputs, num_ticks: int) -> dict:
        """Time every launch shape of this handle's path on num_ticks ticks of
        ``inputs`` (None, numpy or CUDA tensor, as for :meth:`run`) and keep the
        fastest; the state returns to tick 0."""
        flags, ptr, keep = 0, None, None
        if inputs is not None:
            if isinstance(inputs, np.ndarray):
                keep = np.ascontiguousarray(inputs, dtype=np.uint32)
                ptr = keep.ctypes.data
            else:
                flags, ptr, keep = RANC_INPUTS_ON_DEVICE, inputs.data_ptr(), inputs
        return ranc_autotune(self.handle, ptr, flags, num_ticks, self.stream.cuda_stream)

    def launch_shape(self, shape: dict | None = None) -> dict:
        """Set (if given) and return the launch shape."""
        if shape is not None:
            ranc_set_launch_shape(self.handle, shape)
        return ranc_get_launch_shape(self.handle)

    def profile(self, enable: bool = True):
        ranc_profile_enable(self.handle, enable)
        return self

    def profile_read(self) -> dict:
        return ranc_profile_read(self.handle)

    def total_counters(self) -> dict:
        tot = dict(emitted=0, routed=0, delivered=0, out=0, events=0)
        for s in range(self.S):
            for k, v in self.counters(s).items():
                tot[k] += v
        return tot


def run_batch(nets, inputs, num_ticks: int, graph: bool = False, persistent: bool = False):
    """Advance several RancNets together (ranc_run_ticks with num_nets > 1):
    per tick one launch per MFMA shape class, or one persistent work-queue
    launch for all MFMA-path nets with ``persistent``, and one integration and
    one routing launch for all plain-path nets. ``inputs``: one entry per net,
    each None or an array as for :meth:`RancNet.run`; the non-None entries must
    be all numpy arrays (host) or all CUDA tensors (device)."""
    flags = (RANC_RUN_GRAPH if graph else 0) | (RANC_BATCH_PERSISTENT if persistent else 0)
    ptrs, keep = [], []
    kinds = set()
    for g, x in zip(nets, inputs):
        if x is None:
            ptrs.append(None)
            continue
        if isinstance(x, np.ndarray):
            a = np.ascontiguousarray(x, dtype=np.uint32)
            assert a.shape[:2] == (g.S, num_ticks), a.shape
            kinds.add("host")
            keep.append(a)
            ptrs.append(a.ctypes.data)
        else:
            assert x.is_cuda and x.is_contiguous() and x.element_size() == 4
            assert tuple(x.shape[:2]) == (g.S, num_ticks), tuple(x.shape)
            kinds.add("device")
            keep.append(x)
            ptrs.append(x.data_ptr())
    if len(kinds) > 1:
        raise ValueError("batch inputs must be all host arrays or all device tensors")
    if kinds == {"device"}:
        flags |= RANC_INPUTS_ON_DEVICE
    stream = nets[0].stream
    ranc_run_ticks([g.handle for g in nets], ptrs, flags, num_ticks, stream.cuda_stream)
    if kinds == {"host"}:
        stream.synchronize()   # host buffers must outlive the staging copies
    return nets


def decode_raster(words: np.ndarray, out_neurons: np.ndarray, tick_begin: int, sample: int,
                  layout: str = "sample") -> np.ndarray:
    """Output-bus spikes of one sample from a bulk raster (as ranc_copy_raster
    writes it: "sample" u32 [T][S][ceil(Nout/32)] or "neuron" u64
    [T][Nout][ceil(S/64)]), int64 [n, 3] rows (tick, core, neuron) sorted by
    (tick, core, neuron), as RancNet.spikes returns them."""
    nout = len(out_neurons)
    if layout == "sample":
        w = np.ascontiguousarray(np.asarray(words).view(np.uint32)[:, sample, :])
        bits = np.unpackbits(w.view(np.uint8), axis=1, bitorder="little")[:, :nout].astype(bool)
    else:
        w = np.asarray(words).view(np.uint64)
        bits = ((w[:, :, sample // 64] >> np.uint64(sample % 64)) & np.uint64(1)).astype(bool)
    t, o = np.nonzero(bits)
    if not len(t):
        return np.zeros((0, 3), np.int64)
    return np.stack([t.astype(np.int64) + tick_begin, out_neurons[o, 0].astype(np.int64),
                     out_neurons[o, 1].astype(np.int64)], axis=1)
