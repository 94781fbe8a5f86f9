"""The count entry point that allocates nothing (kc_count_noalloc), through the C
ABI, against kc_count on the same handle: two calls in a row, the second on a
smaller graph, at every k; with scratch-tier roots (lowered workgroup cap and
natural out-degrees above the LDS limit), with and without the staged cache."""
import numpy as np
import pytest

from graphgen import small as S
from paper_1403_0734_amd import kc as K

from gpu_util import announce, device_graph

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _lib():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    K.load()


def noalloc(h, k):
    import torch
    out = torch.full((2,), -1, dtype=torch.int64, device="cuda:0")
    K.kc_count_noalloc(h, k, out.data_ptr())
    torch.cuda.synchronize()
    v = out.cpu().numpy().view(np.uint64)
    return int(v[0]), int(v[1])


def prepared(el):
    h = device_graph(el)
    K.kc_count(h, 3)  # builds the degree queue and the staged cache (allocating call)
    return h


@pytest.mark.parametrize("cache", ["1", "0"])
@pytest.mark.parametrize("cap", [0, 72])
def test_noalloc_matches_kc_count(monkeypatch, cap, cache):
    monkeypatch.setenv("KC_STAGE_CACHE", cache)
    K.kc_set_tuning(wg_dmax=cap)
    try:
        # a larger graph, then a smaller one (every tier; the first has scratch-tier
        # roots at any cap: out-degree 1401 is above what LDS holds)
        for el, ks in [(S.hub_bipartite(1400, 1401, 0.05, 3), range(3, 7)),
                       (S.planted_small(400, 0.02, [list(range(0, 60, 2)), list(range(100, 190, 3))], 4), range(3, 9)),
                       (S.random_graph(150, 0.6, 2), range(3, 9))]:
            h = prepared(el)
            for k in ks:
                announce(f"noalloc cap={cap} cache={cache} {el.name} k={k}")
                got = noalloc(h, k)
                assert got == (K.kc_count(h, k), 0), (el.name, k, got)
                assert noalloc(h, k) == got  # the array keeps the last call's contents: cleared per call
            K.kc_graph_destroy(h)
    finally:
        K.kc_set_tuning(defaults=True)


def test_noalloc_needs_a_prepared_handle():
    h = device_graph(S.complete(10))
    with pytest.raises(K.KcError) as e:
        noalloc(h, 4)
    assert e.value.status == K.KC_ESTATE
    K.kc_count(h, 3)
    assert noalloc(h, 4) == (210, 0)
    for bad in (2, K.KC_KMAX + 1):
        with pytest.raises(K.KcError) as e:
            noalloc(h, bad)
        assert e.value.status == K.KC_EINVAL
    with pytest.raises(K.KcError) as e:
        K.kc_count_noalloc(h, 4, None)
    assert e.value.status == K.KC_EINVAL
    K.kc_graph_destroy(h)
