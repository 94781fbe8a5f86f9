"""Helpers for the GPU tests: move an edge list to the device and build a libkc
graph through the C ABI (the binding only marshals pointers)."""
import sys

import numpy as np

from paper_1403_0734_amd import kc as K


def torch_dev():
    import torch
    return torch, torch.device("cuda:0")


def announce(what: str):
    print(f"[gpu] {what}", flush=True)
    sys.stdout.flush()


def device_graph(el, orient=True):
    torch, dev = torch_dev()
    src = torch.from_numpy(el.src.view(np.int32).copy()).to(dev) if el.m_in else torch.zeros(1, dtype=torch.int32, device=dev)
    dst = torch.from_numpy(el.dst.view(np.int32).copy()).to(dev) if el.m_in else torch.zeros(1, dtype=torch.int32, device=dev)
    stream = torch.cuda.current_stream().cuda_stream
    h = K.kc_graph_create(src.data_ptr(), dst.data_ptr(), el.m_in, el.n, True, stream)
    torch.cuda.synchronize()
    if orient:
        K.kc_orient(h)
    return h


def per_root(h, n, k, with_work=False):
    torch, dev = torch_dev()
    c = torch.zeros(n, dtype=torch.int64, device=dev)
    w = torch.zeros(n, dtype=torch.int64, device=dev) if with_work else None
    K.kc_count_per_root(h, k, c.data_ptr(), w.data_ptr() if w is not None else None)
    torch.cuda.synchronize()
    cc = c.cpu().numpy().view(np.uint64)
    ww = w.cpu().numpy().view(np.uint64) if w is not None else None
    return cc, ww


def oriented(h, n, m):
    torch, dev = torch_dev()
    optr = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    ocol = torch.zeros(max(m, 1), dtype=torch.int32, device=dev)
    r2i = torch.zeros(n, dtype=torch.int32, device=dev)
    K.kc_get_oriented(h, optr.data_ptr(), ocol.data_ptr(), r2i.data_ptr())
    torch.cuda.synchronize()
    return (optr.cpu().numpy().view(np.uint64), ocol.cpu().numpy().view(np.uint32)[:m],
            r2i.cpu().numpy().view(np.uint32))


def csr(h, n, m):
    torch, dev = torch_dev()
    rp = torch.zeros(n + 1, dtype=torch.int64, device=dev)
    col = torch.zeros(max(2 * m, 1), dtype=torch.int32, device=dev)
    deg = torch.zeros(n, dtype=torch.int32, device=dev)
    K.kc_get_csr(h, rp.data_ptr(), col.data_ptr(), deg.data_ptr())
    torch.cuda.synchronize()
    return (rp.cpu().numpy().view(np.uint64), col.cpu().numpy().view(np.uint32)[:2 * m],
            deg.cpu().numpy().view(np.uint32))
