"""tc_count_batch_noalloc (scratch in the library's static device array)
against tc_count_batch (caller workspace): T, |H| and the levels of every
graph equal, element by element, on two calls in a row, the second with a
smaller batch (the shared array keeps the first call's contents); and the
host-side refusals (TC_VALIDATE, a batch beyond the array) before any device
work."""
import ctypes

import numpy as np
import pytest

import graphgen
import oracle

pytestmark = pytest.mark.gpu


def _both(b):
    import paper_2210_00389_amd as tc
    ref = tc.count_batch(b, return_levels=True)
    got = tc.count_batch(b, return_levels=True, noalloc=True)
    G = b.num_graphs
    return ([x[:G].cpu().numpy() for x in (ref.triangles, ref.h_count)] + [ref.levels.cpu().numpy()],
            [x[:G].cpu().numpy() for x in (got.triangles, got.h_count)] + [got.levels.cpu().numpy()])


def test_noalloc_matches_workspace_call_twice():
    import torch
    import paper_2210_00389_amd as tc
    big = graphgen.batch_mix(96, seed_base=31, n_max=16384)
    small = [graphgen.complete(9), graphgen.wheel(40), graphgen.cycle(11)] + \
        graphgen.batch_mix(8, seed_base=77, n_max=2048)
    for k, graphs in enumerate((big, small)):
        print(f"case: noalloc call {k} ({len(graphs)} graphs)", flush=True)
        b = tc.Batch.from_graphs(graphs)
        ref, got = _both(b)
        for r, g in zip(ref, got):
            assert np.array_equal(r, g), k
        if k == 1:  # the small batch against the oracle as well
            want = [oracle.triangle_count(oracle.from_graph(g)) for g in graphs]
            assert got[0].tolist() == want
    torch.cuda.synchronize()


def test_noalloc_refusals_before_device_work():
    import torch
    import paper_2210_00389_amd as tc
    from paper_2210_00389_amd import _lib
    lib = _lib.load()
    scratch = lib.tc_noalloc_scratch_bytes()
    assert scratch == 32 << 20
    b = tc.Batch.from_graphs([graphgen.complete(5)])
    with pytest.raises(tc.TcError) as e:
        tc.count_batch(b, noalloc=True, validate=True)
    assert e.value.status == -1
    # a batch whose scratch exceeds the array: refused on the host (the
    # pointers are valid, the sizes are only declared)
    t = torch.zeros(1, dtype=torch.int64, device="cuda")
    tb = _lib.TcBatch(4096, 1 << 30, 1 << 31, b.vbase.data_ptr(), b.row_offsets.data_ptr(), b.cols.data_ptr(), 64)
    rc = lib.tc_count_batch_noalloc(ctypes.byref(tb), None, 0, ctypes.c_void_p(t.data_ptr()), None, None, None)
    assert rc == -8 and "scratch" in lib.tc_last_error().decode()
    assert lib.tc_workspace_bytes(_lib.OP_COUNT_BATCH, 1 << 30, 1 << 31, 4096) > scratch
    torch.cuda.synchronize()
