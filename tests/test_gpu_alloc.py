"""The map's device memory through a caller's allocator (smki_set_allocator):
torch's caching allocator (the binding's default) and hipMalloc give the same
map bit for bit; a failing allocator makes the insert return SMKI_E_OOM and
leaves the map as it was."""
import ctypes as C

import numpy as np
import pytest

import scenes
from gpu_cases import compare_map, cuda, oracle_map_of

pytestmark = pytest.mark.gpu


def _bits(m):
    ijk, a = m.export()
    return ijk.cpu().numpy(), a.cpu().numpy().view(np.uint32)


def test_torch_allocator_and_hipmalloc_give_the_same_map():
    import torch
    from paper_1909_04631_amd import SemanticMap
    sc = scenes.make_config(0)
    p = sc.params
    s = sc.scans[0]
    maps = []
    for alloc in ("torch", None):
        m = SemanticMap.from_params(p, allocator=alloc, initial_blocks=16)   # grows in the inserts
        for part in (slice(0, 700), slice(700, None)):
            m.insert_scan(cuda(s.xyz[part]), cuda(s.label[part]), s.origin, p.free_step)
        torch.cuda.synchronize()
        maps.append(m)
    a, b = _bits(maps[0]), _bits(maps[1])
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    compare_map(maps[0], oracle_map_of(sc), p.K)


def test_failing_allocator_reports_oom_and_leaves_the_map_unchanged():
    import torch
    from paper_1909_04631_amd import SemanticMap, SmkiError, _lib
    sc = scenes.make_config(0)
    p = sc.params
    s = sc.scans[0]
    m = SemanticMap.from_params(p, allocator=None, initial_blocks=16)
    m.insert_scan(cuda(s.xyz[:300]), cuda(s.label[:300]), s.origin, p.free_step)
    torch.cuda.synchronize()
    before = _bits(m)
    calls = []

    def _alloc(nbytes, ctx):
        calls.append(int(nbytes))
        return None            # out of memory

    def _release(ptr, ctx):
        raise AssertionError("nothing was allocated through this allocator")

    cb = (_lib.ALLOC_FN(_alloc), _lib.RELEASE_FN(_release))
    _lib.check(_lib.lib().smki_set_allocator(m._h, cb[0], cb[1], None), "smki_set_allocator")
    with pytest.raises(SmkiError) as e:
        m.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)   # needs more room
    assert e.value.status == -2 and calls
    after = _bits(m)
    assert np.array_equal(before[0], after[0]) and np.array_equal(before[1], after[1])
    # back to hipMalloc: the same insert now succeeds
    _lib.check(_lib.lib().smki_set_allocator(m._h, _lib.ALLOC_FN(), _lib.RELEASE_FN(), None),
               "smki_set_allocator")
    m.insert_scan(cuda(s.xyz), cuda(s.label), s.origin, p.free_step)
    torch.cuda.synchronize()
    compare_map(m, oracle_map_of(sc, scans=[scenes.Scan(s.xyz[:300], s.label[:300], s.origin),
                                            s]), p.K)
