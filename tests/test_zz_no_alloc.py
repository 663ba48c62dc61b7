"""The allocation-free entry point qoc_hess_many_dev_noalloc against qoc_hess_many_dev, through
the C ABI: two calls in a row on the static workspace (the second with a smaller input), each
compared with the allocating entry point's results (same kernels, same launch shapes); an
oversized request is refused with nothing written."""
import sys

import numpy as np
import pytest

from paper_2505_00529_amd import inputs, qoc

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _rel(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _run(p, count, thetas_np, entry):
    import torch

    P = p.P
    th = torch.tensor(thetas_np, dtype=torch.float64, device="cuda").contiguous()
    c = torch.full((count,), 7.0, dtype=torch.float64, device="cuda")
    g = torch.full((count, P), 7.0, dtype=torch.float64, device="cuda")
    h = torch.full((count, P, P), 7.0, dtype=torch.float64, device="cuda")
    st = getattr(qoc.lib(), entry)(p.handle, count, th.data_ptr(), c.data_ptr(), g.data_ptr(), h.data_ptr())
    assert st == qoc.QOC_OK, (entry, st, qoc.lib().qoc_last_error(p.handle))
    p.sync()
    return c.cpu().numpy(), g.cpu().numpy(), h.cpu().numpy()


def _compare(p, thetas_np, label):
    count = thetas_np.shape[0]
    cs, gs, hs = _run(p, count, thetas_np, "qoc_hess_many_dev_noalloc")
    ca, ga, ha = _run(p, count, thetas_np, "qoc_hess_many_dev")
    for i in range(count):
        e = (_rel(cs[i], ca[i]), _rel(gs[i], ga[i]), _rel(hs[i], ha[i]))
        _say(f"  {label} theta {i}: static vs allocating dC={e[0]:.1e} dg={e[1]:.1e} dH={e[2]:.1e}")
        assert max(e) < TOL
    assert np.all(np.isfinite(hs))


def test_noalloc_matches_allocating_entry_point_twice():
    import torch

    torch.cuda.set_device(0)
    _say("no-alloc: molecule n=36 nt=1200, 3 thetas, then tiny n=4 nt=500, 1 theta")
    w = inputs.make_workload("molecule", nt=1200)
    p = qoc.problem_from_workload(w)
    p.set_stream(torch.cuda.current_stream().cuda_stream)
    _compare(p, inputs.draw_thetas(w.p, 3, 61), "first call")
    p.close()
    # second call, smaller input, on another handle: the workspace keeps the first call's data
    w2 = inputs.make_workload("tiny")
    q = qoc.problem_from_workload(w2)
    q.set_stream(torch.cuda.current_stream().cuda_stream)
    _compare(q, inputs.draw_thetas(w2.p, 1, 62), "second call")
    q.close()


def test_noalloc_refuses_oversized_workspace():
    import torch

    torch.cuda.set_device(0)
    # n = 64, nt = 4000: about 0.4 GB of eigen-data per theta, above the 256 MiB workspace
    w = inputs.make_workload("warm")
    p = qoc.problem_from_workload(w)
    P = p.P
    th = torch.zeros(1, P, dtype=torch.float64, device="cuda")
    c = torch.full((1,), 7.0, dtype=torch.float64, device="cuda")
    g = torch.full((1, P), 7.0, dtype=torch.float64, device="cuda")
    h = torch.full((1, P, P), 7.0, dtype=torch.float64, device="cuda")
    st = qoc.lib().qoc_hess_many_dev_noalloc(p.handle, 1, th.data_ptr(), c.data_ptr(), g.data_ptr(), h.data_ptr())
    msg = qoc.lib().qoc_last_error(p.handle).decode()
    _say(f"  oversized: status {st}: {msg}")
    assert st == qoc.QOC_ERR_UNSUPPORTED and "static scratch" in msg
    p.sync()
    assert torch.all(c == 7.0) and torch.all(g == 7.0) and torch.all(h == 7.0)
    p.close()
