"""GPU parity of the grouped execution (grouped launches in a HIP graph)
against the per-instance launches and the FP64 oracle."""
import os

import numpy as np
import pytest
import torch

from paper_2312_13170_amd import synth
from gpu_util import TOL_FP32, dev, empty, host, normwise, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def li():
    from paper_2312_13170_amd import li as mod
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    mod.li_init()
    return mod


class Batch:
    """Device buffers of a batch; C / cov / means reset from host copies."""

    def __init__(self, li, b, inplace_every=0):
        self.li = li
        self.gemm = []
        self.cov = []
        self.problems = []
        for d in b.gemm:
            A, B, C0 = dev(d["A"]), dev(d["B"]), dev(d["C"])
            C = C0.clone()
            self.gemm.append((d, A, B, C0, C))
            self.problems.append(li.make_problem(li.LI_PROBLEM_GEMM, d["M"], d["N"], d["K"], d["alpha"],
                                                 d["beta"], A, B, C))
        for t, d in enumerate(b.cov):
            X0 = dev(d["data"])
            X = X0.clone()
            inplace = inplace_every and t % inplace_every == 0
            Y = X if inplace else empty(X.shape, fill=float("nan"))
            mean = empty((d["M"],), torch.float64, fill=float("nan"))
            cov = empty((d["M"], d["M"]), fill=float("nan"))
            self.cov.append((d, X0, X, Y, mean, cov, inplace))
            self.problems.append(li.make_problem(li.LI_PROBLEM_COVARIANCE, d["M"], d["N"], 0, 1.0, 0.0, X,
                                                 None, cov, Y, mean))

    def reset(self):
        for d, A, B, C0, C in self.gemm:
            C.copy_(C0)
        for d, X0, X, Y, mean, cov, inplace in self.cov:
            X.copy_(X0)
            if not inplace:
                Y.fill_(float("nan"))
            mean.fill_(float("nan"))
            cov.fill_(float("nan"))
        torch.cuda.synchronize()

    def results(self):
        torch.cuda.synchronize()
        g = [host(C) for (_, _, _, _, C) in self.gemm]
        c = [(host(Y), host(mean), host(cov)) for (_, _, _, Y, mean, cov, _) in self.cov]
        return g, c


def small_batch(seed, n):
    b = synth.batch_inputs(seed, n_gemm=0, n_cov=0)
    sizes = synth.loguniform_sizes(seed, "sz", 3 * n, lo=1, hi=300)
    for t in range(n):
        M, N, K = (int(x) for x in sizes[3 * t: 3 * t + 3])
        b.gemm.append(dict(kind="gemm", M=M, N=N, K=K, alpha=1.5, beta=1.2,
                           A=synth.uniform_pm1(seed, "a%d" % t, (M, K)),
                           B=synth.uniform_pm1(seed, "b%d" % t, (K, N)),
                           C=synth.uniform_pm1(seed, "c%d" % t, (M, N))))
        Nc = max(N, 2)
        b.cov.append(dict(kind="cov", M=M, N=Nc, data=synth.uniform_pm1(seed, "x%d" % t, (Nc, M))))
    return b


def check_against_oracle(orc, batch, g, c, idx_g, idx_c):
    for i in idx_g:
        d = batch.gemm[i][0]
        ref = orc.gemm(d["A"], d["B"], d["C"], alpha=d["alpha"], beta=d["beta"])
        assert normwise(g[i], ref) < TOL_FP32, ("gemm", i, d["M"], d["N"], d["K"])
    for i in idx_c:
        d = batch.cov[i][0]
        rY, rmean, rcov = orc.covariance(d["data"])
        Y, mean, cov = c[i]
        assert np.allclose(mean, rmean, rtol=1e-12, atol=1e-13), ("cov mean", i)
        assert normwise(Y, rY) < 1e-7, ("cov data", i)
        assert normwise(cov, rcov) < TOL_FP32, ("cov", i, d["M"], d["N"])
        assert np.array_equal(cov, cov.T)


def test_small_batch_all_instances(li, orc):
    say("grouped small batch")
    b = small_batch(61, 40)
    batch = Batch(li, b, inplace_every=3)
    plan = li.li_group_plan_create(batch.problems)
    batch.reset()
    plan.launch()
    g, c = batch.results()
    check_against_oracle(orc, batch, g, c, range(len(g)), range(len(c)))
    # per-instance launches (same tile shapes) give bitwise the same results
    batch.reset()
    plan.launch_loop()
    g2, c2 = batch.results()
    for x, y in zip(g, g2):
        assert np.array_equal(x, y)
    for (y1, m1, c1), (y2, m2, c2_) in zip(c, c2):
        assert np.array_equal(y1, y2) and np.array_equal(m1, m2) and np.array_equal(c1, c2_)
    plan.close()


@pytest.mark.parametrize("persist", ["0", "1"])
def test_every_class_and_schedule(li, orc, persist):
    # each shape class forced for both problem kinds, on the dispatched and
    # on the resident-grid schedule: every instance against the oracle and
    # bitwise equal to the per-instance launches
    b = small_batch(62, 24)
    batch = Batch(li, b, inplace_every=4)
    n = li.li_tune_num_candidates(li.LI_KERNEL_GROUPED_GEMM)
    assert n == li.li_tune_num_candidates(li.LI_KERNEL_GROUPED_COV) and n >= 2
    old = os.environ.get("LI_GROUPED_PERSIST")
    try:
        os.environ["LI_GROUPED_PERSIST"] = persist
        for cls in range(n):
            say("grouped class", cls, "persist", persist)
            li.li_tune_force(li.LI_KERNEL_GROUPED_GEMM, cls)
            li.li_tune_force(li.LI_KERNEL_GROUPED_COV, cls)
            plan = li.li_group_plan_create(batch.problems)
            batch.reset()
            plan.launch()
            g, c = batch.results()
            check_against_oracle(orc, batch, g, c, range(len(g)), range(len(c)))
            batch.reset()
            plan.launch_loop()
            g2, c2 = batch.results()
            for x, y in zip(g, g2):
                assert np.array_equal(x, y), cls
            for (y1, m1, c1), (y2, m2, c2_) in zip(c, c2):
                assert np.array_equal(y1, y2) and np.array_equal(m1, m2) and np.array_equal(c1, c2_), cls
            plan.close()
    finally:
        li.li_tune_force(li.LI_KERNEL_GROUPED_GEMM, -1)
        li.li_tune_force(li.LI_KERNEL_GROUPED_COV, -1)
        if old is None:
            os.environ.pop("LI_GROUPED_PERSIST", None)
        else:
            os.environ["LI_GROUPED_PERSIST"] = old


def test_grouped_1024_instances(li, orc):
    say("grouped 512 GEMM + 512 covariance instances")
    b = synth.workload("batch_512_512")
    batch = Batch(li, b)
    plan = li.li_group_plan_create(batch.problems)
    assert plan.flops > 1e10
    batch.reset()
    plan.launch_loop()
    g_ref, c_ref = batch.results()
    # several replays of the graph, with eager work and synchronisation between
    for rep in range(3):
        say("  replay", rep)
        batch.reset()
        plan.launch()
        g, c = batch.results()
        for i, (x, y) in enumerate(zip(g, g_ref)):
            assert np.array_equal(x, y), ("gemm", i)
        for i, ((y1, m1, c1), (y2, m2, c2)) in enumerate(zip(c, c_ref)):
            assert np.array_equal(m1, m2) and np.array_equal(y1, y2) and np.array_equal(c1, c2), ("cov", i)
    say("  oracle check of all %d instances" % (len(g) + len(c)))
    check_against_oracle(orc, batch, g, c, range(len(g)), range(len(c)))
    plan.close()


def test_empty_and_degenerate_plans(li):
    say("grouped empty plan")
    plan = li.li_group_plan_create([])
    plan.launch()
    torch.cuda.synchronize()
    assert plan.flops == 0.0
    plan.close()
    say("grouped degenerate problems")
    C = empty((4, 5), fill=2.0)
    probs = [li.make_problem(li.LI_PROBLEM_GEMM, 4, 5, 0, 1.5, 0.5, None, None, C),
             li.make_problem(li.LI_PROBLEM_GEMM, 0, 5, 7, 1.5, 0.5, None, None, None)]
    plan = li.li_group_plan_create(probs)
    plan.launch()
    assert np.all(host(C) == 1.0)
    plan.close()
