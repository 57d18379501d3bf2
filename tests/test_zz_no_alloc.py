"""The allocation-free entry point (mp_vec_dot_noalloc) against mp_vec_dot, through the C ABI.

Two calls in a row, the second on a smaller input: each result equals the allocating
entry point's bit for bit (same kernels, same summation order), and neither the library's
reserved bytes nor torch's allocator move during the calls.
"""
import numpy as np
import pytest

import fixtures as F

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.mark.parametrize("dtype", ["f32", "f64"])
def test_noalloc_dot_matches_dot(dtype):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1101_3615_amd as M
    w = F.tiny(n=16, nb=4, nt=10, ns=1, nr=2, dtype=dtype)
    P = M.Problem.from_spec(w)
    tdt = torch.float32 if dtype == "f32" else torch.float64
    big = 3_000_001
    a = torch.from_numpy(F.normal_field((big,), 401, np.float64)).to("cuda:0", tdt)
    b = torch.from_numpy(F.normal_field((big,), 402, np.float64)).to("cuda:0", tdt)
    out = torch.zeros(2, dtype=torch.float64, device="cuda:0")
    ref_big = P.dot(a, b)                      # allocates its partials on first use
    ref_small = P.dot(a[:1000], b[:1000])
    torch.cuda.synchronize()
    reserved = P.stats()["bytes_reserved"]
    torch_bytes = torch.cuda.memory_allocated()
    got = []
    for n in (big, 1000):
        P.dot_noalloc(a[:n], b[:n], out)
        torch.cuda.synchronize()
        got.append(float(out[0].item()))
    assert P.stats()["bytes_reserved"] == reserved
    assert torch.cuda.memory_allocated() == torch_bytes
    assert got[0] == ref_big and got[1] == ref_small
    an, bn = a.double().cpu().numpy(), b.double().cpu().numpy()
    assert abs(got[0] - float(np.dot(an, bn))) <= 1e-10 * float(np.sum(np.abs(an * bn)))
    P.dot_noalloc(a[:0], b[:0], out)              # n = 0 writes 0
    torch.cuda.synchronize()
    assert float(out[0].item()) == 0.0
    from paper_1101_3615_amd import _lib as L
    rc = P._lib.mp_vec_dot_noalloc(P._ctx, -1, None, None, None, None)
    assert rc == L.MP_EINVAL
