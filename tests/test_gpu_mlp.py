"""Device warm-start network (BF16 matrix-core products, FP32 accumulation) against the CPU
reference evaluated in FP64 with BF16 rounding at the same points."""
import sys

import numpy as np
import pytest

from oracle import mlp_ref as R
from paper_2505_00529_amd import qoc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _cos(a, b):
    return float(np.dot(a, b) / (np.linalg.norm(a) * np.linalg.norm(b)))


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - b) / np.linalg.norm(b))


SHAPES = [
    ("ragged", 20, 40, 24, 37),       # no dimension a multiple of 16
    ("tiny", 3, 5, 2, 1),
    ("warm-start", 128, 512, 64, 256),
]


@pytest.mark.parametrize("name,n_in,h,n_out,batch", SHAPES, ids=[s[0] for s in SHAPES])
def test_mlp_forward_backward_against_reference(name, n_in, h, n_out, batch):
    import torch

    rng = np.random.Generator(np.random.PCG64(100 + n_in))
    p = R.init_params(n_in, h, n_out, seed=n_in)
    x = rng.normal(size=(batch, n_in)).astype(np.float32)
    t = (0.3 * rng.normal(size=(batch, n_out))).astype(np.float32)
    _say(f"mlp {name}: {n_in}->{h}->{h}->{n_out}, batch {batch}")
    net = qoc.Mlp(n_in, h, n_out, max_batch=batch)
    net.set_params(p)
    xd = torch.from_numpy(x).cuda()
    td = torch.from_numpy(t).cuda()
    yd = torch.empty((batch, n_out), dtype=torch.float32, device="cuda")
    ld = torch.zeros((), dtype=torch.float32, device="cuda")
    net.forward(batch, xd.data_ptr(), yd.data_ptr())
    net.loss_grad(batch, xd.data_ptr(), td.data_ptr(), ld.data_ptr())
    net.sync()
    y = yd.cpu().numpy().astype(np.float64)
    g = net.get_grads().astype(np.float64)
    loss_ref, g_ref, f = R.loss_and_grads(p, x, t, n_in, h, n_out, mirror_bf16=True)
    ey = _rel(y, f["y"])
    el = abs(ld.item() - loss_ref) / loss_ref
    parts = R.unpack(g, n_in, h, n_out)
    parts_ref = R.unpack(g_ref, n_in, h, n_out)
    cos = [_cos(a.ravel(), b.ravel()) for a, b in zip(parts, parts_ref)]
    eg = [_rel(a, b) for a, b in zip(parts, parts_ref)]
    _say(f"  y rel {ey:.2e}  loss rel {el:.2e}  grad cos min {min(cos):.6f}  grad rel max {max(eg):.2e}")
    assert ey < 1e-2 and el < 1e-2
    assert min(cos) > 0.999 and max(eg) < 5e-2
    net.close()


def test_mlp_train_step_applies_adam_to_device_gradients():
    import torch

    n_in, h, n_out, batch = 24, 48, 8, 33
    rng = np.random.Generator(np.random.PCG64(7))
    p = R.init_params(n_in, h, n_out, seed=5)
    x = torch.from_numpy(rng.normal(size=(batch, n_in)).astype(np.float32)).cuda()
    t = torch.from_numpy(rng.normal(size=(batch, n_out)).astype(np.float32)).cuda()
    net = qoc.Mlp(n_in, h, n_out, max_batch=64)
    net.set_params(p)
    pr = p.astype(np.float64)
    m = np.zeros_like(pr)
    v = np.zeros_like(pr)
    lr = 1e-3
    losses = []
    ld = torch.zeros((), dtype=torch.float32, device="cuda")
    for step in range(1, 4):
        net.train_step(batch, x.data_ptr(), t.data_ptr(), lr, loss_ptr=ld.data_ptr())
        net.sync()
        losses.append(ld.item())
        g = net.get_grads().astype(np.float64)
        pr, m, v = R.adam_step(pr, g, m, v, step, lr)
        dev = net.get_params().astype(np.float64)
        err = np.abs(dev - pr).max()
        _say(f"  adam step {step}: loss {losses[-1]:.6f} max |param - reference| {err:.2e}")
        assert err < 1e-6
        pr = dev     # continue from the device's FP32 values
    assert losses[-1] < losses[0]


def test_mlp_rejects_bad_batch():
    import torch

    net = qoc.Mlp(4, 8, 2, max_batch=4)
    x = torch.zeros((8, 4), dtype=torch.float32, device="cuda")
    y = torch.zeros((8, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(qoc.QocError):
        net.forward(5, x.data_ptr(), y.data_ptr())
    with pytest.raises(qoc.QocError):
        net.forward(0, x.data_ptr(), y.data_ptr())
    with pytest.raises(ValueError):
        net.set_params(np.zeros(3, np.float32))
    net.close()
