"""Batched instances (qpat_batch): several contexts on their own streams
advanced by one call give exactly the results of calling them one by one,
and those match the oracle."""
import numpy as np
import pytest
import torch

from gpu_util import GpuProblem, dev, host, need_gpu, oracle_of, assert_close
from qpat_inputs import make_problem, probe_vectors

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    need_gpu()


def instances():
    from paper_1512_02796_amd import qpat
    out = []
    for name, over in (("T8", {}), ("T12", {}), ("T24", {"n_ill": 5}), ("C4", {"n": 20, "n_ill": 7, "id": 4999})):
        P = make_problem(name, **over)
        m = P.mesh
        st = torch.cuda.Stream()
        ctx = qpat.Context(dev(m.coords), dev(m.tets, torch.int32), dev(m.bfaces, torch.int32),
                           opts=qpat.default_opts(pcg_rtol=1e-12), stream=st)
        ctx.set_sources(dev(P.phi_src))
        s, t = probe_vectors(P.cfg["id"], P.n_ill, m.N)
        out.append((P, ctx, dev(s), dev(t)))
    return out


def test_batch_equals_one_by_one():
    from paper_1512_02796_amd import qpat
    inst = instances()
    ctxs = [c for _, c, _, _ in inst]
    H = [torch.empty(P.n_ill * P.mesh.N, dtype=torch.float64, device="cuda") for P, _, _, _ in inst]
    qpat.batch(ctxs, "forward", in0=[dev(P.kappa) for P, *_ in inst], in1=[dev(P.mu) for P, *_ in inst], out0=H)
    JS = [torch.empty_like(h) for h in H]
    JT = [torch.empty(2 * P.mesh.N, dtype=torch.float64, device="cuda") for P, *_ in inst]
    infos = qpat.batch(ctxs, "pair", in0=[s for *_, s, _ in inst], out0=JS, in1=[t for *_, t in inst], out1=JT)
    torch.cuda.synchronize()
    for (P, ctx, s, t), js, jt, info in zip(inst, JS, JT, infos):
        h1 = torch.empty_like(js)
        ctx.forward(dev(P.kappa), dev(P.mu), None, h1)
        a = torch.empty_like(js)
        b = torch.empty_like(jt)
        ctx.jvp(s, a)
        ctx.vjp(t, b)
        torch.cuda.synchronize()
        assert torch.equal(a, js) and torch.equal(b, jt)
        assert info["n_solves"] >= 2 * P.n_ill and info["relres_max"] <= 1e-12
        assert len(info["rhs_iters"]) == info["n_solves"]
        if P.mesh.N <= 20000:     # the oracle's sparse LU at these sizes takes seconds
            g, lin = oracle_of(P)
            assert_close(host(h1).reshape(P.n_ill, -1), lin.h, 1e-10, f"h n={P.mesh.n}")
            sh, th = host(s), host(t).reshape(P.n_ill, -1)
            assert_close(host(js).reshape(P.n_ill, -1), lin.jvp(sh), 1e-10, f"J s n={P.mesh.n}")
            assert_close(host(jt), lin.vjp(th), 1e-10, f"J^T t n={P.mesh.n}")
    for c in ctxs:
        c.close()


def test_batch_rejects_shared_stream():
    from paper_1512_02796_amd import qpat
    G = GpuProblem("T4")
    with pytest.raises(qpat.QpatError):
        qpat.batch([G.ctx, G.ctx], "lsqr_step")
