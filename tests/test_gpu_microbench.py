"""The device microbenchmarks count what they claim: every LDS and global
atomic add of 1 lands (exact integer totals), and the copy copies."""
import pytest

pytestmark = pytest.mark.gpu


def test_microbenchmarks_count_their_operations():
    import ctypes as C
    import torch
    from paper_1608_05238_amd import _lib as L
    lib = L.load()
    d = torch.device("cuda", 0)
    s = C.c_void_p(torch.cuda.current_stream(d).cuda_stream)
    nblk, iters = 40, 24
    sink = torch.empty(nblk, dtype=torch.float64, device=d)
    clk = torch.zeros(4, dtype=torch.int64, device=d)
    for kind, per in ((L.MB_LDS_ADD_F64, 1), (L.MB_LDS_ADD_F32, 1), (L.MB_LDS_ADD_U64, 1), (L.MB_LDS_ADD_U32, 1),
                      (L.MB_LDS_ADD_F64_ROW33, 33), (L.MB_LDS_ADD_U64_ROW33, 33), (L.MB_LDS_ADD_U64_PRE, 8)):
        for block, lds in ((256, 4096), (256, 96 * 1024), (1024, 144 * 1024)):   # the last: the transport's shape
            assert lib.mb_lds_atomics(kind, lds, block, nblk, iters, 5, sink.data_ptr(), clk.data_ptr(), s) == 0
            torch.cuda.synchronize()
            assert torch.all(sink == block * iters * per), (kind, lds, sink[:4])
            c = clk.cpu().tolist()
            assert c[1] > c[0] and c[3] > c[2]
    n = 1000
    buf = torch.zeros(n, dtype=torch.float64, device=d)
    assert lib.mb_global_atomics_f64(buf.data_ptr(), n, 16, 10, 1, s) == 0
    torch.cuda.synchronize()
    assert float(buf.sum()) == 16 * 256 * 10
    rows = torch.zeros(500 * 33, dtype=torch.float64, device=d)
    assert lib.mb_global_atomics_rows_f64(rows.data_ptr(), 500, 33, 16, 40, 2, s) == 0
    torch.cuda.synchronize()
    assert float(rows.sum()) == 16 * 256 * 40 and float(rows.min()) >= 0
    a = torch.arange(4 * 3000, dtype=torch.float32, device=d)
    b = torch.zeros_like(a)
    assert lib.mb_copy(a.data_ptr(), b.data_ptr(), 3000, s) == 0
    fs = torch.empty(8 * 256, dtype=torch.float32, device=d)
    assert lib.mb_fma_f32(fs.data_ptr(), 8, 100, clk.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert bool(torch.isfinite(fs).all())
