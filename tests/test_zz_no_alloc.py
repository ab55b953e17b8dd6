"""tr_mttkrp_noalloc (the allocation-free variant of tr_mttkrp: partials in
the library's file-scope device array) against tr_mttkrp with a caller
workspace, through the C ABI: two calls in a row, the second on a smaller
problem, in FP64 and FP32.  Both run the same kernels with the same work
split, so the results must agree bit for bit (the FP64 parity bound, 1e-10
entry by entry, is the stated bar; equality is what is expected).  A
problem whose partials exceed the array is refused before any device work.
"""

import numpy as np
import pytest

import workloads as W
from parity import dev

pytestmark = pytest.mark.gpu


def _pair(trlib, dims, ranks, dt, seed, accumulate):
    import torch
    cores, X = W.random_tr_problem(dims, ranks, seed, noise=0.1)
    tdt = torch.float64 if dt == "f64" else torch.float32
    code = 0 if dt == "f64" else 1
    Xt = torch.from_numpy(np.asfortranarray(X)).to(tdt).cuda()
    ct = [torch.from_numpy(np.asfortranarray(G)).to(tdt).cuda() for G in cores]
    wsb = trlib.tr_workspace_bytes(list(dims), list(ranks), dt)
    ws = torch.empty(wsb, dtype=torch.uint8, device="cuda")
    st_ = torch.cuda.current_stream().cuda_stream
    out = []
    for n in range(len(dims)):
        d = ranks[n] * ranks[(n + 1) % len(dims)]
        base = torch.randn((dims[n], d), dtype=torch.float64, device="cuda")
        P1 = base.clone()
        P2 = base.clone()
        trlib.tr_mttkrp(list(dims), list(ranks), code, n, Xt.data_ptr(),
                        [c.data_ptr() for c in ct], P1.data_ptr(), accumulate, ws.data_ptr(), wsb,
                        st_)
        trlib.tr_mttkrp_noalloc(list(dims), list(ranks), code, n, Xt.data_ptr(),
                                [c.data_ptr() for c in ct], P2.data_ptr(), accumulate, st_)
        torch.cuda.synchronize()
        a, b = P1.cpu().numpy(), P2.cpu().numpy()
        print(f"[noalloc {dims} {dt} n={n} acc={accumulate}] dev {dev(b, a):.2e} "
              f"equal {np.array_equal(a, b)}", flush=True)
        out.append((a, b))
    return out


@pytest.mark.parametrize("dt", ["f64", "f32"])
def test_noalloc_matches_workspace_entry(trlib, dt):
    # first call: 256 x 256 x 20 (the streaming batch shape), then a smaller,
    # ragged order-4 problem that reuses the same array
    for dims, ranks, acc in [((256, 256, 20), (8, 8, 8), 0), ((13, 9, 7, 5), (2, 3, 4, 2), 1)]:
        for a, b in _pair(trlib, dims, ranks, dt, 3, acc):
            assert dev(b, a) < 1e-10
            assert np.array_equal(a, b)


def test_noalloc_rejects_oversized(trlib):
    import torch
    assert trlib.tr_mttkrp_noalloc_max_bytes() == 16 << 20
    # 64^3 x 2000 with TR-ranks 16, temporal mode: five chunks of partials of
    # 2000 x 256 doubles, 20.5 MB
    dims, ranks = (64, 64, 64, 2000), (16, 16, 16, 16)
    X = torch.zeros(8, dtype=torch.float64, device="cuda")      # never read
    cores = [torch.zeros(8, dtype=torch.float64, device="cuda") for _ in range(4)]
    P = torch.zeros(8, dtype=torch.float64, device="cuda")
    with pytest.raises(trlib.TRError) as e:
        trlib.tr_mttkrp_noalloc(list(dims), list(ranks), 0, 3, X.data_ptr(),
                                [c.data_ptr() for c in cores], P.data_ptr(), 0,
                                torch.cuda.current_stream().cuda_stream)
    assert e.value.status == "TR_ERR_UNSUPPORTED"
