"""The single-launch 2D periodic solve (one workgroup holds the half spectrum).

* every operator it takes (psi, GRAD, CURL of a scalar, NABLA), PS and FD2
  eigenvalues, FP32 and FP64, against the oracle element by element;
* the same problem on the three general passes (HP_SMALL2D=0) agrees;
* the plan really is one pass, and sizes beyond the kernel's LDS budget keep
  the general passes;
* replays of a captured graph equal the eager solve.
"""
import numpy as np
import pytest

from gpu_util import TOL, case_input, gpu_solve, oracle_solve, rel_l2, rel_max

pytestmark = pytest.mark.gpu

LO = [0.0, -0.5]
HI = [1.0, 1.3]
# sizes whose input spectrum and one output spectrum fit (every operator), and
# sizes where only the in-place plain solve fits
WITH_DERIV = [("f64", [64, 64]), ("f32", [64, 64]), ("f32", [64, 128]), ("f32", [128, 64])]
PSI_ONLY = [("f64", [64, 128]), ("f64", [128, 64]), ("f32", [128, 128]), ("f32", [64, 256]),
            ("f32", [256, 64])]
CASES = [(p, nc, d) for p, nc in WITH_DERIV for d in ("none", "grad", "curl", "nabla")] + \
        [(p, nc, "none") for p, nc in PSI_ONLY]


def check(got, ref, prec, what):
    l2, mx = TOL[prec]
    e2, em = rel_l2(got, ref), rel_max(got, ref)
    assert e2 <= l2 and em <= mx, f"{what}: rel-L2 {e2:.3e} rel-max {em:.3e}"


def n_passes(nc, kernel, diff, prec):
    import torch
    from paper_2301_01145_amd import Solver
    dtype = torch.float32 if prec == "f32" else torch.float64
    s = Solver("periodic", "staggered", nc, LO, HI, kernel=kernel, diff=diff, dtype=dtype)
    n = s.passes()
    s.close()
    return n


@pytest.mark.parametrize("prec,nc,diff", CASES)
@pytest.mark.parametrize("kernel", ["ps", "fd2"])
def test_small2d_matches_oracle(prec, nc, diff, kernel):
    print(f"small2d {prec} {nc} {diff} {kernel}", flush=True)
    assert n_passes(nc, kernel, diff, prec) == 1
    f, _ = case_input("periodic", "staggered", nc, 1, False, prec, seed=61)
    got, gd = gpu_solve("periodic", "staggered", nc, LO, HI, f, kernel, diff, prec, 1, None)
    ref, rd = oracle_solve("periodic", "staggered", nc, LO, HI, f, kernel, diff, None)
    check(got, ref, prec, "psi")
    assert len(gd) == len(rd)
    for a in range(len(gd)):
        check(gd[a], rd[a], prec, f"{diff} {a}")


@pytest.mark.parametrize("prec,nc,diff", [("f64", [64, 64], "none"), ("f64", [64, 64], "grad"),
                                          ("f64", [64, 64], "curl"), ("f64", [64, 64], "nabla"),
                                          ("f32", [128, 64], "grad"), ("f32", [256, 64], "none")])
def test_small2d_matches_general(prec, nc, diff, monkeypatch):
    f, _ = case_input("periodic", "staggered", nc, 1, False, prec, seed=67)
    one, od = gpu_solve("periodic", "staggered", nc, LO, HI, f, "ps", diff, prec, 1, None)
    monkeypatch.setenv("HP_SMALL2D", "0")
    assert n_passes(nc, "ps", diff, prec) == 3
    gen, gd = gpu_solve("periodic", "staggered", nc, LO, HI, f, "ps", diff, prec, 1, None)
    check(one, gen, prec, "psi")
    for a in range(len(gd)):
        check(od[a], gd[a], prec, f"{diff} {a}")


@pytest.mark.parametrize("prec,nc,diff", [("f64", [128, 128], "none"), ("f32", [128, 256], "none"),
                                          ("f32", [128, 128], "grad"), ("f64", [64, 128], "curl"),
                                          ("f64", [48, 64], "none"), ("f64", [64, 60], "none")])
def test_small2d_not_taken(prec, nc, diff):
    # half spectrum beyond the LDS budget, or a length without a wavefront FFT
    assert n_passes(nc, "ps", diff, prec) == 3
    f, _ = case_input("periodic", "staggered", nc, 1, False, prec, seed=71)
    got, _ = gpu_solve("periodic", "staggered", nc, LO, HI, f, "ps", diff, prec, 1, None)
    ref, _ = oracle_solve("periodic", "staggered", nc, LO, HI, f, "ps", diff, None)
    check(got, ref, prec, "psi")


def test_small2d_graph_replay():
    import torch
    from paper_2301_01145_amd import Solver
    side = torch.cuda.Stream()
    rng = np.random.default_rng(73)
    with torch.cuda.stream(side):
        s = Solver("periodic", "staggered", [64, 64], kernel="ps", diff="grad", dtype=torch.float64)
        f = torch.as_tensor(rng.normal(size=(64, 64)), device="cuda")
        psi, der = s.bind(f)
        s.run()
    torch.cuda.synchronize()
    eager = [t.cpu().numpy().copy() for t in list(psi) + list(der)]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=side):
        s.run()
    torch.cuda.synchronize()
    for rep in range(3):
        for t in list(psi) + list(der):
            t.fill_(float("nan"))
        junk = torch.randn(1 << 20, device="cuda") * 2.0  # eager work between replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for i, t in enumerate(list(psi) + list(der)):
            assert np.array_equal(t.cpu().numpy(), eager[i]), (rep, i)
        del junk
    s.close()
