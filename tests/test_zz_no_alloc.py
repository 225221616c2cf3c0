"""qpat_misfit_noalloc: the allocation-free variant of qpat_misfit, whose
partial sums live in the library's file-scope device array. Its result must
equal qpat_misfit's on two calls in a row, the second with a smaller problem
(another context on the same GPU, so the shared array is reused with fewer
partial sums), and on a repeat of the first."""
import numpy as np
import pytest
import torch

from gpu_util import GpuProblem, oracle_of, data_of, dev, need_gpu

pytestmark = pytest.mark.gpu


def test_misfit_noalloc_matches_misfit():
    need_gpu()
    cases = []
    for name in ("T24", "T8"):            # the second call's problem is smaller
        G = GpuProblem(name)
        G.forward()
        g, lin = oracle_of(G.P)
        chi, W = data_of(G.P, lin)
        cases.append((G, dev(chi), dev(W)))
    for G, chi, W in cases + cases[:1]:
        out = torch.full((1,), -1.0, dtype=torch.float64, device="cuda")
        G.ctx.misfit_noalloc(chi, W, out)
        ref = G.ctx.misfit(chi, W)          # the existing entry point (synchronises)
        got = float(out.item())
        assert np.isfinite(got) and ref > 0.0
        assert abs(got - ref) <= 1e-15 * ref, (got, ref)
    # before any forward solve the variant refuses, like qpat_misfit
    from paper_1512_02796_amd import qpat
    H = GpuProblem("T4")
    out = torch.zeros(1, dtype=torch.float64, device="cuda")
    with pytest.raises(qpat.QpatError) as e:
        H.ctx.misfit_noalloc(torch.zeros(H.n_ill * H.N, dtype=torch.float64, device="cuda"),
                             torch.ones(H.n_ill * H.N, dtype=torch.float64, device="cuda"), out)
    assert e.value.status == qpat.QPAT_ERR_STATE
