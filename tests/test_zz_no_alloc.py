"""The allocation-free compaction entry point (gv_compact3_noalloc) against
the existing compaction entry (gv_debug_step, GV_DBG_COMPACT), through the C
ABI, on device buffers: two calls in a row, the second with a smaller input,
must give the same queues and counts; sizes beyond the scratch limit and bad
blocks are rejected before anything is enqueued.

Device buffers come from the HIP runtime the library itself links (through
ctypes), so the test runs the same in a fresh process and after the other
GPU tests."""
import ctypes as C

import numpy as np
import pytest

import gv_inputs

pytestmark = pytest.mark.gpu

H2D, D2H = 1, 2


class _Hip:
    def __init__(self):
        self.lib = C.CDLL("libamdhip64.so.7")
        self.lib.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.lib.hipFree.argtypes = [C.c_void_p]
        self.lib.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.lib.hipDeviceSynchronize.argtypes = []

    def alloc(self, nbytes):
        p = C.c_void_p()
        assert self.lib.hipMalloc(C.byref(p), max(nbytes, 1)) == 0
        return p.value

    def put(self, arr):
        a = np.ascontiguousarray(arr)
        p = self.alloc(a.nbytes)
        assert self.lib.hipMemcpy(p, a.ctypes.data, a.nbytes, H2D) == 0
        return p

    def get(self, p, dtype, n):
        out = np.zeros(n, dtype=dtype)
        assert self.lib.hipMemcpy(out.ctypes.data, p, out.nbytes, D2H) == 0
        return out

    def free(self, *ps):
        for p in ps:
            self.lib.hipFree(p)


def _run(gv, hip, codes, block):
    n = len(codes)
    dc = hip.put(codes.astype(np.int8))
    di = hip.put(np.full(max(9 * n, 1), -7, dtype=np.int32))
    dn = hip.put(np.full(4, 99, dtype=np.uint32))
    gv.compact3_noalloc(dc, n, block, di, dn, None)
    assert hip.lib.hipDeviceSynchronize() == 0
    counts = hip.get(dn, np.uint32, 4)
    idx = hip.get(di, np.int32, 9 * n).reshape(3, 3 * n) if n else np.zeros((3, 0), np.int32)
    hip.free(dc, di, dn)
    return counts, idx


def test_noalloc_compaction_equals_the_debug_entry():
    import paper_2005_00949_amd as gv
    eng = gv.Engine(gv_inputs.slab_calorimeter(1), precision=gv.P64)
    hip = _Hip()
    rng = np.random.default_rng(77)
    for n, block in ((1_000_003, 256), (70_001, 64), (3, 128)):
        codes = rng.integers(-1, 3, size=(n, 3)).astype(np.int8)
        codes[rng.random(n) < 0.3, 1:] = -1
        ref = eng.debug_compact(codes, block=block)
        counts, idx = _run(gv, hip, codes, block)
        print(f"\n[noalloc n={n} block={block}] counts {counts.tolist()}")
        assert counts[3] == 0
        for q in range(3):
            assert counts[q] == len(ref[q])
            assert np.array_equal(idx[q, : counts[q]], ref[q])
    counts, _ = _run(gv, hip, np.zeros((0, 3), np.int8), 64)
    assert counts.tolist() == [0, 0, 0, 0]


def test_noalloc_rejects_sizes_beyond_the_scratch():
    import paper_2005_00949_amd as gv
    gv.load()
    hip = _Hip()
    p = hip.put(np.zeros(16, dtype=np.int32))
    with pytest.raises(gv.GvError):
        gv.compact3_noalloc(p, (1 << 24) + 1, 256, p, p, None)
    with pytest.raises(gv.GvError):
        gv.compact3_noalloc(p, 10, 32, p, p, None)
    with pytest.raises(gv.GvError):
        gv.compact3_noalloc(0, 10, 64, p, p, None)
    assert hip.get(p, np.int32, 16).tolist() == [0] * 16
    hip.free(p)
