"""Thin ctypes binding of libkc (include/kc.h).

Argument marshalling only: every step of the counting path runs in the HIP
library.  Device buffers and streams may come from torch (``tensor.data_ptr()``,
``torch.cuda.current_stream().cuda_stream``); nothing else from torch is used.
The binding raises when libkc.so is missing: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libkc.so")

KC_OK, KC_EINVAL, KC_ESTATE, KC_ENOMEM, KC_EOVERFLOW, KC_EDEVICE = 0, -1, -2, -3, -4, -5
KC_COLOR_PER_ROOT, KC_COLOR_GLOBAL = 0, 1
KC_SCHED_DEGREE, KC_SCHED_LEARNED, KC_SCHED_EDGES = 0, 1, 2
KC_KMAX = 10
KC_MLP_PARAMS = 1377

# every symbol include/kc.h declares
EXPORTS = [
    "kc_graph_create", "kc_orient", "kc_count", "kc_count_colored", "kc_count_pair_sampled", "kc_count_per_root",
    "kc_count_batch", "kc_set_schedule", "kc_train_schedule", "kc_graph_info", "kc_get_csr",
    "kc_get_oriented", "kc_last_timings", "kc_graph_destroy", "kc_status_str",
    "kc_set_tuning", "kc_get_tuning", "kc_autotune", "kc_last_tier_timings", "kc_count_noalloc",
    "kc_predict_work", "kc_mlp_step", "kc_last_stage_timings", "kc_count_per_node",
]


class KcError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class kc_estimate(ctypes.Structure):
    _fields_ = [("raw", ctypes.c_uint64), ("estimate", ctypes.c_double), ("estimate_u64", ctypes.c_uint64),
                ("estimate_fits_u64", ctypes.c_int32), ("scale_exponent", ctypes.c_int32)]


class kc_tuning(ctypes.Structure):
    _fields_ = [("wave_dmax", ctypes.c_int32), ("wg_blocks_per_cu", ctypes.c_int32),
                ("wave_blocks_per_cu", ctypes.c_int32), ("queue_chunk_div", ctypes.c_int32),
                ("wg_dmax", ctypes.c_int32), ("local_bits", ctypes.c_int32), ("wg_waves", ctypes.c_int32)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libkc.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"libkc.so not found at {path}: build it with `python -m paper_1403_0734_amd.build`")
    # PyTorch-ROCm ships its own HIP runtime under the same soname.  Loaded after
    # libkc.so, it would be a second runtime in the process (device pointers and
    # streams of one are unknown to the other); loaded first, libkc.so binds to it.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    P, i32, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_uint32, ctypes.c_uint64
    sig = {
        "kc_graph_create": (i32, [P, P, u64, u32, i32, P, ctypes.POINTER(P)]),
        "kc_orient": (i32, [P]),
        "kc_count": (i32, [P, i32, ctypes.POINTER(u64)]),
        "kc_count_colored": (i32, [P, i32, u32, u64, i32, ctypes.POINTER(kc_estimate)]),
        "kc_count_pair_sampled": (i32, [P, i32, ctypes.c_double, u64, ctypes.POINTER(kc_estimate)]),
        "kc_count_per_root": (i32, [P, i32, P, P]),
        "kc_count_per_node": (i32, [P, i32, P]),
        "kc_count_noalloc": (i32, [P, i32, P]),
        "kc_predict_work": (i32, [P, i32, P, P]),
        "kc_mlp_step": (i32, [P, P, P, i32, ctypes.c_float, P, P, u32, P, ctypes.POINTER(ctypes.c_float), P]),
        "kc_count_batch": (i32, [P, u32, i32, P]),
        "kc_set_schedule": (i32, [P, i32, ctypes.c_char_p]),
        "kc_train_schedule": (i32, [P, u32, i32, i32, u64, ctypes.c_char_p, ctypes.POINTER(ctypes.c_float)]),
        "kc_graph_info": (i32, [P, ctypes.POINTER(u32), ctypes.POINTER(u64), ctypes.POINTER(u32)]),
        "kc_get_csr": (i32, [P, P, P, P]),
        "kc_get_oriented": (i32, [P, P, P, P]),
        "kc_last_timings": (i32, [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                  ctypes.POINTER(ctypes.c_float)]),
        "kc_graph_destroy": (None, [P]),
        "kc_status_str": (ctypes.c_char_p, [i32]),
        "kc_set_tuning": (i32, [ctypes.POINTER(kc_tuning)]),
        "kc_get_tuning": (i32, [ctypes.POINTER(kc_tuning)]),
        "kc_autotune": (i32, [P, u32, i32, ctypes.c_char_p, ctypes.POINTER(kc_tuning)]),
        "kc_last_tier_timings": (i32, [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                       ctypes.POINTER(ctypes.c_float)]),
        "kc_last_stage_timings": (i32, [P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float),
                                        ctypes.POINTER(ctypes.c_float)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(status: int, what: str = ""):
    if status != KC_OK:
        msg = load().kc_status_str(status).decode()
        raise KcError(status, f"{what}: {msg}" if what else msg)


def _ptr(x) -> int | None:
    """Device or host address of a torch tensor / numpy array / int."""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    if hasattr(x, "data_ptr"):
        return x.data_ptr()
    if hasattr(x, "ctypes"):
        return x.ctypes.data
    raise TypeError(f"cannot take the address of {type(x)}")


def kc_graph_create(src, dst, m_in: int, n: int, src_on_device: bool, stream=None) -> int:
    h = ctypes.c_void_p()
    check(load().kc_graph_create(_ptr(src), _ptr(dst), m_in, n, int(src_on_device), stream, ctypes.byref(h)),
          "kc_graph_create")
    return h.value


def kc_orient(g: int):
    check(load().kc_orient(g), "kc_orient")


def kc_count(g: int, k: int) -> int:
    q = ctypes.c_uint64()
    check(load().kc_count(g, k, ctypes.byref(q)), f"kc_count(k={k})")
    return q.value


def kc_count_colored(g: int, k: int, c: int, seed: int, scheme: int = KC_COLOR_PER_ROOT) -> kc_estimate:
    e = kc_estimate()
    check(load().kc_count_colored(g, k, c, seed, scheme, ctypes.byref(e)), "kc_count_colored")
    return e


def kc_count_pair_sampled(g: int, k: int, p: float, seed: int) -> kc_estimate:
    e = kc_estimate()
    check(load().kc_count_pair_sampled(g, k, float(p), seed, ctypes.byref(e)), "kc_count_pair_sampled")
    return e


def kc_count_per_root(g: int, k: int, dev_counts, dev_work=None):
    check(load().kc_count_per_root(g, k, _ptr(dev_counts), _ptr(dev_work)), "kc_count_per_root")


def kc_count_per_node(g: int, k: int, dev_counts):
    """Per-node clique-membership counts into device uint64[n] (by original id)."""
    check(load().kc_count_per_node(g, k, _ptr(dev_counts)), "kc_count_per_node")


def kc_count_noalloc(g: int, k: int, dev_out):
    """Enqueue an exact count that allocates nothing; dev_out: device uint64[2]
    (q_k, overflow flag), valid once the handle's stream reaches this call."""
    check(load().kc_count_noalloc(g, k, _ptr(dev_out)), f"kc_count_noalloc(k={k})")


def kc_count_batch(gs, k: int) -> list:
    arr = (ctypes.c_void_p * len(gs))(*gs)
    out = (ctypes.c_uint64 * len(gs))()
    check(load().kc_count_batch(arr, len(gs), k, out), "kc_count_batch")
    return list(out)


def kc_set_schedule(g: int, policy: int, weights_path: str | None = None):
    check(load().kc_set_schedule(g, policy, weights_path.encode() if weights_path else None), "kc_set_schedule")


def kc_train_schedule(gs, k: int, epochs: int, seed: int, weights_path: str) -> float:
    arr = (ctypes.c_void_p * len(gs))(*gs)
    loss = ctypes.c_float()
    check(load().kc_train_schedule(arr, len(gs), k, epochs, seed, weights_path.encode(), ctypes.byref(loss)),
          "kc_train_schedule")
    return loss.value


def kc_set_tuning(wave_dmax=64, wg_blocks_per_cu=0, wave_blocks_per_cu=8, queue_chunk_div=8, wg_dmax=0,
                  local_bits=128, wg_waves=0, defaults=False):
    if defaults:
        check(load().kc_set_tuning(None), "kc_set_tuning")
        return
    t = kc_tuning(wave_dmax, wg_blocks_per_cu, wave_blocks_per_cu, queue_chunk_div, wg_dmax, local_bits, wg_waves)
    check(load().kc_set_tuning(ctypes.byref(t)), "kc_set_tuning")


def kc_get_tuning() -> dict:
    t = kc_tuning()
    check(load().kc_get_tuning(ctypes.byref(t)), "kc_get_tuning")
    return {f: getattr(t, f) for f, _ in kc_tuning._fields_}


def kc_autotune(gs, k: int, cache_path: str | None = None) -> dict:
    arr = (ctypes.c_void_p * len(gs))(*gs)
    t = kc_tuning()
    check(load().kc_autotune(arr, len(gs), k, cache_path.encode() if cache_path else None, ctypes.byref(t)),
          "kc_autotune")
    return {f: getattr(t, f) for f, _ in kc_tuning._fields_}


def kc_predict_work(g: int, k: int, dev_pred, dev_feat=None):
    """The scheduler MLP's predicted log(1 + work) per root (device float[n], by
    original id) and optionally its raw features (device float[n][8])."""
    check(load().kc_predict_work(g, k, _ptr(dev_pred), _ptr(dev_feat)), f"kc_predict_work(k={k})")


def kc_mlp_step(params, adam_m, adam_v, step: int, lr: float, x, t, count: int, grad=None, stream=None) -> float:
    """One gradient + Adam step of the scheduler MLP on device samples; returns the
    batch loss before the update."""
    loss = ctypes.c_float()
    check(load().kc_mlp_step(_ptr(params), _ptr(adam_m), _ptr(adam_v), step, float(lr), _ptr(x), _ptr(t), count,
                             _ptr(grad), ctypes.byref(loss), stream), "kc_mlp_step")
    return loss.value


def kc_graph_info(g: int):
    n, m, d = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint32()
    check(load().kc_graph_info(g, ctypes.byref(n), ctypes.byref(m), ctypes.byref(d)), "kc_graph_info")
    return n.value, m.value, d.value


def kc_get_csr(g: int, row_ptr=None, col=None, deg=None):
    check(load().kc_get_csr(g, _ptr(row_ptr), _ptr(col), _ptr(deg)), "kc_get_csr")


def kc_get_oriented(g: int, optr=None, ocol=None, rank2id=None):
    check(load().kc_get_oriented(g, _ptr(optr), _ptr(ocol), _ptr(rank2id)), "kc_get_oriented")


def kc_last_timings(g: int):
    a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
    check(load().kc_last_timings(g, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "kc_last_timings")
    return a.value, b.value, c.value


def kc_last_tier_timings(g: int):
    a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
    check(load().kc_last_tier_timings(g, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "kc_last_tier_timings")
    return a.value, b.value, c.value


def kc_last_stage_timings(g: int):
    a, b, c = ctypes.c_float(), ctypes.c_float(), ctypes.c_float()
    check(load().kc_last_stage_timings(g, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)), "kc_last_stage_timings")
    return a.value, b.value, c.value


def kc_graph_destroy(g: int):
    if g:
        load().kc_graph_destroy(g)


class Graph:
    """Owning wrapper around a kc_graph handle (marshalling only)."""

    def __init__(self, src, dst, n: int, stream=None):
        on_dev = hasattr(src, "is_cuda") and bool(src.is_cuda)
        m_in = int(src.numel() if hasattr(src, "numel") else len(src))
        self._keep = (src, dst)
        self.h = kc_graph_create(src, dst, m_in, n, on_dev, stream)
        self._keep = None

    def orient(self):
        kc_orient(self.h)
        return self

    def count(self, k: int) -> int:
        return kc_count(self.h, k)

    def count_colored(self, k: int, c: int, seed: int, scheme: int = KC_COLOR_PER_ROOT) -> kc_estimate:
        return kc_count_colored(self.h, k, c, seed, scheme)

    def info(self):
        return kc_graph_info(self.h)

    def close(self):
        if getattr(self, "h", None):
            kc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()
