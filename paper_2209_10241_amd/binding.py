"""Thin ctypes binding of libhomotif.so (names follow include/homotif.h).

Argument marshalling only: every step of the counting runs in the HIP
library.  Device memory and streams come from PyTorch; outputs are torch
tensors on the current device.  Importing this module does not need a GPU;
calling a counting entry point does.  When the library has not been built,
every entry point raises ``LibraryMissing``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhomotif.so")

HM_OK = 0
HM_EINVAL = -1
HM_EUNSUPPORTED = -2
HM_ENOMEM = -3
HM_EDEVICE = -4
HM_EINTERNAL = -5
HM_MEM_HOST = 0
HM_MEM_DEVICE = 1
HM_OPT_BITSET_MAX_NODES = 1
HM_OPT_SAMPLE_CHUNK_SCALE = 2
HM_OPT_ONE_PASS_MAX_EDGES = 3
HM_OPT_HUB_MIN_DEGREE = 4
HM_OPT_DEDUP_TAG_BITS = 5
HM_ALLOC_PROPORTIONAL = 0
HM_ALLOC_PAPER = 1
HM_NULL_STUBS = 0
HM_NULL_CONFIG = 1

_ERROR_NAMES = {HM_EINVAL: "HM_EINVAL", HM_EUNSUPPORTED: "HM_EUNSUPPORTED", HM_ENOMEM: "HM_ENOMEM",
                HM_EDEVICE: "HM_EDEVICE", HM_EINTERNAL: "HM_EINTERNAL"}


class LibraryMissing(ImportError):
    pass


class HMError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{_ERROR_NAMES.get(code, code)}: {message}")
        self.code = code


_lib = None

_vp = ctypes.c_void_p
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_int = ctypes.c_int
_dbl = ctypes.c_double

# name -> (restype, argtypes)
SIGNATURES = {
    "hm_last_error": (ctypes.c_char_p, []),
    "hm_version": (ctypes.c_char_p, []),
    "hm_num_classes": (_int, [_int]),
    "hm_class_info": (_int, [_int, _int, _vp, _vp, _vp]),
    "hm_pattern_class": (_int, [_int, _u32, _vp]),
    "hm_graph_create": (_int, [_vp, _vp, _u64, _u64, _u32, _int, _vp, _vp]),
    "hm_graph_destroy": (_int, [_vp]),
    "hm_graph_stats": (_int, [_vp, _vp]),
    "hm_graph_export": (_int, [_vp, _int, _vp]),
    "count_exact": (_int, [_vp, _int, _vp, _vp]),
    "count_exact_many": (_int, [_int, _vp, _vp, _vp, _vp, _vp, _int, _int, _vp, _int, _vp]),
    "count_exact_noalloc": (_int, [_vp, _int, _vp, _vp]),
    "count_baseline": (_int, [_vp, _int, _vp, _vp, _vp]),
    "hm_sample_sizes": (_int, [_vp, _int, _dbl, _int, _vp]),
    "hm_sample_sizes_for": (_int, [_int, _vp, _dbl, _int, _vp]),
    "hm_sample_draw": (_int, [_vp, _int, _dbl, _u64, _int, _vp, _vp, _vp, _vp]),
    "count_sampled": (_int, [_vp, _int, _dbl, _u64, _int, _vp, _vp, _vp]),
    "count_sampled5": (_int, [_vp, _dbl, _u64, _u64, _vp, _vp, _vp, _vp, _vp]),
    "count_sampled5_indices": (_int, [_vp, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _u64, _u64, _vp, _vp, _vp, _vp, _vp]),
    "hm_order5_sizes": (_int, [_vp, _vp, _vp]),
    "count_sampled_sizes": (_int, [_vp, _int, _u64, _u64, _u64, _u64, _vp, _vp, _vp]),
    "hm_stratum_search": (_int, [_vp, _int, _u64, _vp, _int, _vp, _int, _int, _u64, _vp, _int, _vp, _dbl, _vp, _vp]),
    "count_sampled_indices": (_int, [_vp, _int, _vp, _u64, _vp, _u64, _vp, _u64, _vp, _vp, _vp]),
    "count_nulls": (_int, [_vp, _int, _int, _u64, _vp, _vp, _vp, _vp]),
    "count_nulls_model": (_int, [_vp, _int, _int, _int, _int, _u64, _vp, _vp, _vp, _vp]),
    "hm_null_export": (_int, [_vp, _u64, _u32, _vp, _vp]),
    "hm_null_export_model": (_int, [_vp, _int, _int, _u64, _u32, _vp, _vp]),
    "hm_motif_profile": (_int, [_vp, _vp, _int, _int, _dbl, _vp, _vp, _vp]),
    "hm_profile_quality": (_int, [_vp, _vp, _int, _vp, _vp]),
    "hm_null_tile_sizes": (_int, [_vp, _vp]),
    "hm_features": (_int, [_vp, _int, _vp, _vp]),
    "hm_contrib": (_int, [_vp, _int, _vp, _vp]),
    "hm_mlp_forward": (_int, [_vp, _vp, _u64, _vp, _vp]),
    "hm_mlp_grad": (_int, [_vp, _vp, _vp, _u64, _vp, _vp]),
    "hm_model_train": (_int, [_vp, _int, _vp, _vp]),
    "hm_model_destroy": (_int, [_vp]),
    "hm_model_params": (_int, [_vp, _vp]),
    "hm_model_loss": (_int, [_vp, _int, _vp]),
    "hm_proposal_probs": (_int, [_vp, _vp, _int, _vp, _vp]),
    "count_sampled_learned": (_int, [_vp, _vp, _int, _dbl, _u64, _vp, _vp, _vp]),
    "count_sampled_weighted_indices": (_int, [_vp, _int, _vp, _vp, _u64, _vp, _vp, _u64, _vp, _vp, _u64, _vp, _vp,
                                              _vp]),
    "hm_set_option": (_int, [_int, ctypes.c_int64]),
    "hm_get_option": (_int, [_int, _vp]),
    "hm_profile_enable": (_int, [_int]),
    "hm_profile_reset": (_int, []),
    "hm_profile_read": (_int, [_int, _vp, _vp, _vp]),
}


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise LibraryMissing(f"{LIB_PATH} is not built (python -m paper_2209_10241_amd.build)")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _check(rc: int) -> int:
    if rc < 0:
        raise HMError(rc, lib().hm_last_error().decode())
    return rc


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def hm_version() -> str:
    return lib().hm_version().decode()


def hm_num_classes(k: int) -> int:
    return _check(lib().hm_num_classes(k))


def hm_class_info(k: int, cls: int):
    canon = ctypes.c_uint32()
    mc = ctypes.c_int()
    cm = ctypes.c_int()
    _check(lib().hm_class_info(k, cls, ctypes.byref(canon), ctypes.byref(mc), ctypes.byref(cm)))
    return canon.value, mc.value, cm.value


def hm_pattern_class(k: int, pattern: int) -> int:
    """Class id of a labelled pattern, -1 when it is not connected."""
    cls = ctypes.c_int()
    _check(lib().hm_pattern_class(k, pattern, ctypes.byref(cls)))
    return cls.value


class Graph:
    """Owner of an ``hm_graph`` handle."""

    def __init__(self, handle: int, n_nodes: int):
        self._h = ctypes.c_void_p(handle)
        self.n_nodes = n_nodes

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise HMError(HM_EINVAL, "graph handle already destroyed")
        return self._h

    def stats(self) -> dict:
        out = (ctypes.c_uint64 * 10)()
        _check(lib().hm_graph_stats(self.handle, out))
        keys = ["n_nodes", "n2", "n3", "n4", "n5plus", "n_input", "singletons", "duplicates", "n_unique",
                "n_unique_members"]
        return dict(zip(keys, [int(x) for x in out]))

    def export(self, j: int) -> np.ndarray:
        n = self.stats()[f"n{j}"]
        out = np.zeros(n * j, dtype=np.uint32)
        _check(lib().hm_graph_export(self.handle, j, out.ctypes.data_as(ctypes.c_void_p)))
        return out.reshape(n, j)

    def close(self):
        if self._h is not None and self._h.value and _lib is not None:
            _lib.hm_graph_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def hm_graph_create(members, offsets, n_nodes: int, stream=None) -> Graph:
    """members/offsets: numpy arrays (host) or CUDA torch tensors (device)."""
    out = ctypes.c_void_p()
    try:
        import torch
        is_dev = isinstance(members, torch.Tensor) and members.is_cuda
    except ImportError:
        is_dev = False
    if is_dev:
        import torch
        members = members.to(torch.int32).contiguous()
        offsets = offsets.to(torch.int64).contiguous()
        n_edges = offsets.numel() - 1
        rc = lib().hm_graph_create(ctypes.c_void_p(members.data_ptr()), ctypes.c_void_p(offsets.data_ptr()),
                                   n_edges, members.numel(), n_nodes, HM_MEM_DEVICE, _stream_ptr(stream),
                                   ctypes.byref(out))
    else:
        m = np.ascontiguousarray(members, dtype=np.uint32)
        o = np.ascontiguousarray(offsets, dtype=np.uint64)
        n_edges = len(o) - 1
        st = _stream_ptr(stream) if _cuda_available() else ctypes.c_void_p(0)
        rc = lib().hm_graph_create(m.ctypes.data_as(ctypes.c_void_p), o.ctypes.data_as(ctypes.c_void_p),
                                   n_edges, len(m), n_nodes, HM_MEM_HOST, st, ctypes.byref(out))
    _check(rc)
    return Graph(out.value, n_nodes)


def _cuda_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except ImportError:
        return False


def count_exact(H: Graph, k: int, out=None, stream=None):
    """Exact per-class counts (int64 torch tensor on the current device)."""
    import torch
    n = hm_num_classes(k)
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device="cuda")
    _check(lib().count_exact(H.handle, k, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def count_exact_many(graphs, k: int, workers: int = 3, out=None, stream=None):
    """Exact per-class counts of many hypergraphs in one call.  graphs: a
    sequence of (members, offsets, n_nodes), members/offsets CUDA torch tensors
    (int32 / int64).  Returns an int64 tensor of len(graphs) x classes."""
    import torch
    n = len(graphs)
    C = hm_num_classes(k)
    if out is None:
        out = torch.empty((n, C), dtype=torch.int64, device="cuda")
    keep = []
    mp, op = (ctypes.c_void_p * max(n, 1))(), (ctypes.c_void_p * max(n, 1))()
    ne, nm = (ctypes.c_uint64 * max(n, 1))(), (ctypes.c_uint64 * max(n, 1))()
    nn = (ctypes.c_uint32 * max(n, 1))()
    seen = {}   # a tensor pair given several times is converted once
    for g, (members, offsets, n_nodes) in enumerate(graphs):
        key = (id(members), id(offsets))
        if key not in seen:
            m = members.to(torch.int32).contiguous()
            o = offsets.to(torch.int64).contiguous()
            keep += [m, o]
            seen[key] = (m.data_ptr(), o.data_ptr(), o.numel() - 1, m.numel())
        mp[g], op[g], ne[g], nm[g] = seen[key]
        nn[g] = n_nodes
    _check(lib().count_exact_many(n, mp, op, ne, nm, nn, HM_MEM_DEVICE, k, ctypes.c_void_p(out.data_ptr()), workers,
                                  _stream_ptr(stream)))
    return out


def count_exact_noalloc(H: Graph, k: int, out=None, stream=None):
    """count_exact without device allocation in the library (graphs with bit rows)."""
    import torch
    if out is None:
        out = torch.empty(hm_num_classes(k), dtype=torch.int64, device="cuda")
    _check(lib().count_exact_noalloc(H.handle, k, ctypes.c_void_p(out.data_ptr()), _stream_ptr(stream)))
    return out


def count_baseline(H: Graph, k: int, out=None, stats=None, stream=None):
    """Exact per-class counts by the projection baseline (Algorithm 1):
    (int64 counts, uint64 [candidates, discarded]) torch tensors on the
    current device."""
    import torch
    n = hm_num_classes(k)
    if out is None:
        out = torch.empty(n, dtype=torch.int64, device="cuda")
    if stats is None:
        stats = torch.empty(2, dtype=torch.int64, device="cuda")
    _check(lib().count_baseline(H.handle, k, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(stats.data_ptr()),
                                _stream_ptr(stream)))
    return out, stats


def hm_profile_enable(on: bool = True) -> None:
    _check(lib().hm_profile_enable(1 if on else 0))


def hm_profile_reset() -> None:
    _check(lib().hm_profile_reset())


def hm_profile_read(max_entries: int = 64) -> dict:
    """{kernel name: (launches, total milliseconds)} since the last reset."""
    names = ctypes.create_string_buffer(64 * max_entries)
    launches = (ctypes.c_uint64 * max_entries)()
    ms = (ctypes.c_double * max_entries)()
    n = _check(lib().hm_profile_read(max_entries, names, launches, ms))
    raw = names.raw
    out = {}
    for i in range(n):
        name = raw[64 * i:64 * (i + 1)].split(b"\0", 1)[0].decode()
        out[name] = (int(launches[i]), float(ms[i]))
    return out


def hm_set_option(option: int, value: int) -> None:
    _check(lib().hm_set_option(option, int(value)))


def hm_get_option(option: int) -> int:
    v = ctypes.c_int64()
    _check(lib().hm_get_option(option, ctypes.byref(v)))
    return v.value


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None and t.numel() else ctypes.c_void_p(0)


def hm_sample_sizes(H: Graph, k: int, fraction: float, allocation: int = HM_ALLOC_PROPORTIONAL):
    out = (ctypes.c_uint64 * 3)()
    _check(lib().hm_sample_sizes(H.handle, k, float(fraction), allocation, out))
    return {2: int(out[0]), 3: int(out[1]), 4: int(out[2])}


def hm_sample_sizes_for(k: int, n_by_size, fraction: float, allocation: int = HM_ALLOC_PROPORTIONAL):
    """Sample sizes from the stratum sizes (|E_2|, |E_3|, |E_4|) alone (host only)."""
    n = (ctypes.c_uint64 * 3)(*[int(x) for x in n_by_size])
    out = (ctypes.c_uint64 * 3)()
    _check(lib().hm_sample_sizes_for(k, n, float(fraction), allocation, out))
    return {2: int(out[0]), 3: int(out[1]), 4: int(out[2])}


def hm_sample_draw(H: Graph, k: int, fraction: float, seed: int, allocation: int = HM_ALLOC_PROPORTIONAL,
                   stream=None) -> dict:
    """Drawn stratum indices {j: uint32 tensor on the device}."""
    import torch
    S = hm_sample_sizes(H, k, fraction, allocation)
    out = {j: torch.empty(S[j], dtype=torch.int32, device="cuda") for j in (2, 3, 4)}
    _check(lib().hm_sample_draw(H.handle, k, float(fraction), int(seed) & (2**64 - 1), allocation,
                                _ptr(out[2]), _ptr(out[3]), _ptr(out[4]), _stream_ptr(stream)))
    return out


def count_sampled(H: Graph, k: int, fraction: float, seed: int, allocation: int = HM_ALLOC_PROPORTIONAL,
                  est=None, raw=None, stream=None):
    """(estimates fp32, raw int64) torch tensors on the current device."""
    import torch
    n = hm_num_classes(k)
    if est is None:
        est = torch.empty(n, dtype=torch.float32, device="cuda")
    if raw is None:
        raw = torch.empty(n, dtype=torch.int64, device="cuda")
    _check(lib().count_sampled(H.handle, k, float(fraction), int(seed) & (2**64 - 1), allocation,
                               ctypes.c_void_p(est.data_ptr()), ctypes.c_void_p(raw.data_ptr()),
                               _stream_ptr(stream)))
    return est, raw


def count_sampled_indices(H: Graph, k: int, samples: dict, est=None, raw=None, stream=None):
    """samples: {j: int tensor/array of stratum indices}; returns (est, raw)."""
    import torch
    n = hm_num_classes(k)
    if est is None:
        est = torch.empty(n, dtype=torch.float32, device="cuda")
    if raw is None:
        raw = torch.empty(n, dtype=torch.int64, device="cuda")
    dev = {}
    for j in (2, 3, 4):
        v = samples.get(j)
        if v is None:
            dev[j] = None
            continue
        t = torch.as_tensor(np.asarray(v) if not isinstance(v, torch.Tensor) else v)
        dev[j] = t.to(device="cuda", dtype=torch.int32).contiguous()
    size = {j: (dev[j].numel() if dev[j] is not None else 0) for j in (2, 3, 4)}
    _check(lib().count_sampled_indices(H.handle, k, _ptr(dev[2]), size[2], _ptr(dev[3]), size[3], _ptr(dev[4]),
                                       size[4], ctypes.c_void_p(est.data_ptr()), ctypes.c_void_p(raw.data_ptr()),
                                       _stream_ptr(stream)))
    return est, raw


def count_nulls(H: Graph, k: int, n_rand: int, seed: int, stream=None):
    """(real int64[C], nulls int64[n_rand, C], z fp32[C]) torch tensors on the current device."""
    import torch
    n = hm_num_classes(k)
    real = torch.empty(n, dtype=torch.int64, device="cuda")
    nulls = torch.empty((n_rand, n), dtype=torch.int64, device="cuda")
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(lib().count_nulls(H.handle, k, n_rand, int(seed) & (2**64 - 1), ctypes.c_void_p(real.data_ptr()),
                             ctypes.c_void_p(nulls.data_ptr()), ctypes.c_void_p(z.data_ptr()), _stream_ptr(stream)))
    return real, nulls, z


def hm_null_export(H: Graph, seed: int, copy: int):
    """(members uint32, offsets uint64) numpy arrays of one null copy."""
    st = H.stats()
    members = np.zeros(max(1, st["n_unique_members"]), dtype=np.uint32)
    offsets = np.zeros(st["n_unique"] + 1, dtype=np.uint64)
    _check(lib().hm_null_export(H.handle, int(seed) & (2**64 - 1), copy, members.ctypes.data_as(ctypes.c_void_p),
                                offsets.ctypes.data_as(ctypes.c_void_p)))
    return members[:st["n_unique_members"]], offsets


def count_nulls_model(H: Graph, k: int, n_rand: int, model: int, sweeps: int, seed: int, stream=None):
    """count_nulls under a chosen null model (HM_NULL_STUBS or HM_NULL_CONFIG)."""
    import torch
    n = hm_num_classes(k)
    real = torch.empty(n, dtype=torch.int64, device="cuda")
    nulls = torch.empty((n_rand, n), dtype=torch.int64, device="cuda")
    z = torch.empty(n, dtype=torch.float32, device="cuda")
    _check(lib().count_nulls_model(H.handle, k, n_rand, model, sweeps, int(seed) & (2**64 - 1),
                                   ctypes.c_void_p(real.data_ptr()), ctypes.c_void_p(nulls.data_ptr()),
                                   ctypes.c_void_p(z.data_ptr()), _stream_ptr(stream)))
    return real, nulls, z


def hm_null_export_model(H: Graph, model: int, sweeps: int, seed: int, copy: int):
    """(members uint32, offsets uint64) numpy arrays of one copy of the chosen null model."""
    st = H.stats()
    members = np.zeros(max(1, st["n_unique_members"]), dtype=np.uint32)
    offsets = np.zeros(st["n_unique"] + 1, dtype=np.uint64)
    _check(lib().hm_null_export_model(H.handle, model, sweeps, int(seed) & (2**64 - 1), copy,
                                      members.ctypes.data_as(ctypes.c_void_p),
                                      offsets.ctypes.data_as(ctypes.c_void_p)))
    return members[:st["n_unique_members"]], offsets


def hm_motif_profile(real, nulls, eps: float = 4.0, stream=None):
    """(delta, sp) float64 tensors: relative abundance against the null rows and its normalised form."""
    import torch
    real = torch.as_tensor(real).to(device="cuda", dtype=torch.float64).contiguous()
    nulls = torch.as_tensor(nulls).to(device="cuda", dtype=torch.float64).contiguous()
    C = real.numel()
    delta = torch.empty(C, dtype=torch.float64, device="cuda")
    sp = torch.empty(C, dtype=torch.float64, device="cuda")
    _check(lib().hm_motif_profile(_ptr(real), _ptr(nulls), nulls.shape[0], C, float(eps), _ptr(delta), _ptr(sp),
                                  _stream_ptr(stream)))
    return delta, sp


def hm_profile_quality(est, exact, stream=None):
    """(rho, MaxAE, MAE) of an estimated profile against the exact one."""
    import torch
    est = torch.as_tensor(est).to(device="cuda", dtype=torch.float64).contiguous()
    exact = torch.as_tensor(exact).to(device="cuda", dtype=torch.float64).contiguous()
    out = torch.empty(3, dtype=torch.float64, device="cuda")
    _check(lib().hm_profile_quality(_ptr(est), _ptr(exact), est.numel(), _ptr(out), _stream_ptr(stream)))
    return tuple(float(x) for x in out.cpu().tolist())


def count_sampled_sizes(H: Graph, k: int, sizes: dict, seed: int, est=None, raw=None, stream=None):
    """Algorithm 4 with sizes[j] draws from stratum j; (est fp32[C], raw int64[C])."""
    import torch
    n = hm_num_classes(k)
    if est is None:
        est = torch.empty(n, dtype=torch.float32, device="cuda")
    if raw is None:
        raw = torch.empty(n, dtype=torch.int64, device="cuda")
    _check(lib().count_sampled_sizes(H.handle, k, int(sizes.get(2, 0)), int(sizes.get(3, 0)), int(sizes.get(4, 0)),
                                     int(seed) & (2**64 - 1), _ptr(est), _ptr(raw), _stream_ptr(stream)))
    return est, raw


def hm_stratum_search(H: Graph, k: int, S: int, ratio3, ratio4, reps: int, seed: int, nulls, exact_profile,
                      eps: float = 4.0, stream=None) -> np.ndarray:
    """Mean Pearson correlation per (ratio3[i], ratio4[j]) cell, as a numpy array [n3, n4]."""
    import torch
    r3 = np.ascontiguousarray(ratio3, dtype=np.float64)
    r4 = np.ascontiguousarray(ratio4 if k == 4 else [0.0], dtype=np.float64)
    nulls = torch.as_tensor(nulls).to(device="cuda", dtype=torch.float64).contiguous()
    prof = torch.as_tensor(exact_profile).to(device="cuda", dtype=torch.float64).contiguous()
    rho = np.zeros((len(r3), len(r4)), dtype=np.float64)
    _check(lib().hm_stratum_search(H.handle, k, int(S), r3.ctypes.data_as(ctypes.c_void_p), len(r3),
                                   r4.ctypes.data_as(ctypes.c_void_p), len(r4), int(reps), int(seed) & (2**64 - 1),
                                   _ptr(nulls), nulls.shape[0], _ptr(prof), float(eps),
                                   rho.ctypes.data_as(ctypes.c_void_p), _stream_ptr(stream)))
    return rho


def hm_order5_sizes(H: Graph, stream=None) -> dict:
    out = (ctypes.c_uint64 * 4)()
    _check(lib().hm_order5_sizes(H.handle, out, _stream_ptr(stream)))
    return {2: int(out[0]), 3: int(out[1]), 4: int(out[2]), 5: int(out[3])}


def _order5_out(capacity):
    import torch
    return (torch.empty(capacity, dtype=torch.int32, device="cuda"),
            torch.empty(capacity, dtype=torch.int64, device="cuda"),
            torch.empty(capacity, dtype=torch.float32, device="cuda"))


def count_sampled5(H: Graph, fraction: float, seed: int, capacity: int = 1 << 20, stream=None):
    """Order-5 Algorithm 4: (canonical uint32 numpy, raw int64 numpy, est float32 numpy), ascending canonical."""
    canon, raw, est = _order5_out(capacity)
    n = ctypes.c_uint64(0)
    _check(lib().count_sampled5(H.handle, float(fraction), int(seed) & (2**64 - 1), capacity, _ptr(canon), _ptr(raw),
                                _ptr(est), ctypes.byref(n), _stream_ptr(stream)))
    k = n.value
    return (canon[:k].cpu().numpy().view(np.uint32), raw[:k].cpu().numpy(), est[:k].cpu().numpy())


def count_sampled5_indices(H: Graph, samples: dict, capacity: int = 1 << 20, stream=None):
    """Order-5 Algorithm 4 on explicit draws {j: indices}, j = 2..5."""
    import torch
    idx = {j: torch.as_tensor(np.asarray(samples.get(j, []), dtype=np.int32)).to("cuda") for j in (2, 3, 4, 5)}
    canon, raw, est = _order5_out(capacity)
    n = ctypes.c_uint64(0)
    _check(lib().count_sampled5_indices(H.handle, _ptr(idx[2]), idx[2].numel(), _ptr(idx[3]), idx[3].numel(),
                                        _ptr(idx[4]), idx[4].numel(), _ptr(idx[5]), idx[5].numel(), capacity,
                                        _ptr(canon), _ptr(raw), _ptr(est), ctypes.byref(n), _stream_ptr(stream)))
    k = n.value
    return (canon[:k].cpu().numpy().view(np.uint32), raw[:k].cpu().numpy(), est[:k].cpu().numpy())


def hm_null_tile_sizes(H: Graph):
    out = (ctypes.c_uint32 * 3)()
    _check(lib().hm_null_tile_sizes(H.handle, out))
    return [int(x) for x in out]


N_PARAMS = 5313


class TrainOpts(ctypes.Structure):
    _fields_ = [("epochs", ctypes.c_int), ("batch", ctypes.c_int), ("lr", ctypes.c_float),
                ("gamma", ctypes.c_float), ("epsilon", ctypes.c_float), ("seed", ctypes.c_uint64)]


def _rows(H: Graph, k: int) -> int:
    st = H.stats()
    return st["n2"] + st["n3"] + (st["n4"] if k == 4 else 0)


def hm_features(H: Graph, k: int, stream=None):
    import torch
    x = torch.empty((_rows(H, k), 16), dtype=torch.float32, device="cuda")
    _check(lib().hm_features(H.handle, k, _ptr(x), _stream_ptr(stream)))
    return x


def hm_contrib(H: Graph, k: int, stream=None):
    import torch
    y = torch.empty(_rows(H, k), dtype=torch.float64, device="cuda")
    _check(lib().hm_contrib(H.handle, k, _ptr(y), _stream_ptr(stream)))
    return y


def hm_mlp_forward(params, x, stream=None):
    import torch
    params = params.to(device="cuda", dtype=torch.float32).contiguous()
    x = x.to(device="cuda", dtype=torch.float32).contiguous()
    out = torch.empty(x.shape[0], dtype=torch.float32, device="cuda")
    _check(lib().hm_mlp_forward(_ptr(params), _ptr(x), x.shape[0], _ptr(out), _stream_ptr(stream)))
    return out


def hm_mlp_grad(params, x, t, stream=None):
    """(gradient [5313], loss) of the mean squared error."""
    import torch
    params = params.to(device="cuda", dtype=torch.float32).contiguous()
    x = x.to(device="cuda", dtype=torch.float32).contiguous()
    t = t.to(device="cuda", dtype=torch.float32).contiguous()
    g = torch.empty(N_PARAMS + 1, dtype=torch.float32, device="cuda")
    _check(lib().hm_mlp_grad(_ptr(params), _ptr(x), _ptr(t), x.shape[0], _ptr(g), _stream_ptr(stream)))
    return g[:N_PARAMS], float(g[N_PARAMS].item())


class Model:
    """Owner of an ``hm_model`` handle (a trained proposal)."""

    def __init__(self, handle: int):
        self._h = ctypes.c_void_p(handle)

    @property
    def handle(self):
        if self._h is None or not self._h.value:
            raise HMError(HM_EINVAL, "model handle already destroyed")
        return self._h

    def params(self) -> np.ndarray:
        out = np.zeros(N_PARAMS, dtype=np.float32)
        _check(lib().hm_model_params(self.handle, out.ctypes.data_as(ctypes.c_void_p)))
        return out

    def loss(self) -> np.ndarray:
        n = _check(lib().hm_model_loss(self.handle, 0, None))
        out = np.zeros(max(n, 1), dtype=np.float32)
        _check(lib().hm_model_loss(self.handle, n, out.ctypes.data_as(ctypes.c_void_p)))
        return out[:n]

    def close(self):
        if self._h is not None and self._h.value and _lib is not None:
            _lib.hm_model_destroy(self._h)
        self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def hm_model_train(H: Graph, k: int, epochs: int = 30, batch: int = 4096, lr: float = 3e-3, gamma: float = 0.7,
                   epsilon: float = 0.1, seed: int = 0) -> Model:
    opts = TrainOpts(epochs, batch, lr, gamma, epsilon, int(seed) & (2**64 - 1))
    out = ctypes.c_void_p()
    _check(lib().hm_model_train(H.handle, k, ctypes.byref(opts), ctypes.byref(out)))
    return Model(out.value)


def hm_proposal_probs(H: Graph, M: Model, k: int, stream=None):
    import torch
    p = torch.empty(_rows(H, k), dtype=torch.float64, device="cuda")
    _check(lib().hm_proposal_probs(H.handle, M.handle, k, _ptr(p), _stream_ptr(stream)))
    return p


def count_sampled_learned(H: Graph, M: Model, k: int, fraction: float, seed: int, stream=None):
    import torch
    n = hm_num_classes(k)
    est = torch.empty(n, dtype=torch.float32, device="cuda")
    raw = torch.empty(n, dtype=torch.int64, device="cuda")
    _check(lib().count_sampled_learned(H.handle, M.handle, k, float(fraction), int(seed) & (2**64 - 1), _ptr(est),
                                       _ptr(raw), _stream_ptr(stream)))
    return est, raw


def count_sampled_weighted_indices(H: Graph, k: int, samples: dict, probs: dict, stream=None):
    """Hansen-Hurwitz estimate: samples {j: indices}, probs {j: probability of each draw}."""
    import torch
    n = hm_num_classes(k)
    est = torch.empty(n, dtype=torch.float32, device="cuda")
    raw = torch.empty(n, dtype=torch.int64, device="cuda")
    idx, pr, size = {}, {}, {}
    for j in (2, 3, 4):
        if samples.get(j) is None or len(samples[j]) == 0:
            idx[j] = pr[j] = None
            size[j] = 0
            continue
        idx[j] = torch.as_tensor(np.asarray(samples[j]), dtype=torch.int32).cuda().contiguous()
        pr[j] = torch.as_tensor(np.asarray(probs[j]), dtype=torch.float64).cuda().contiguous()
        size[j] = idx[j].numel()
    _check(lib().count_sampled_weighted_indices(H.handle, k, _ptr(idx[2]), _ptr(pr[2]), size[2], _ptr(idx[3]),
                                                _ptr(pr[3]), size[3], _ptr(idx[4]), _ptr(pr[4]), size[4], _ptr(est),
                                                _ptr(raw), _stream_ptr(stream)))
    return est, raw
