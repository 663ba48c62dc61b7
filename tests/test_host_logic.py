"""Host-side logic that needs no GPU: warm-start feature and parameter packing, cost
agreement classification, and the benchmark's counter-summary lookup."""
import json
import os

import numpy as np

import bench
from oracle import mlp_ref as R
from paper_2505_00529_amd import warmstart as W


def test_target_features_are_real_and_imaginary_parts():
    t = np.array([[1 + 2j, 3 - 4j], [0.5j, -1.0]])
    x = W.target_features(t)
    assert x.dtype == np.float32 and x.shape == (2, 4)
    assert np.array_equal(x, np.array([[1, 3, 2, -4], [0, -1, 0.5, 0]], np.float32))


def test_init_params_packing_matches_reference_layout():
    n_in, h, n_out = 6, 10, 4
    p = W.init_params(n_in, h, n_out, seed=3)
    assert p.dtype == np.float32 and p.size == h * n_in + h + h * h + h + n_out * h + n_out
    W1, b1, W2, b2, W3, b3 = R.unpack(p, n_in, h, n_out)
    # uniform(-1/sqrt(fan_in), 1/sqrt(fan_in)) per layer
    for mat, bias, fan_in in ((W1, b1, n_in), (W2, b2, h), (W3, b3, h)):
        bound = 1 / np.sqrt(fan_in)
        assert np.abs(mat).max() <= bound and np.abs(bias).max() <= bound
    assert np.array_equal(W.init_params(n_in, h, n_out, seed=3), p)


def test_cost_agreement_counts_matches_and_misses():
    plain = np.array([1.0, 2.0, 3.0, 4.0])
    warm = np.array([1.0 + 5e-9, 2.0 - 1e-6, 3.0 + 1e-3, 4.0])
    r = W.compare(plain, warm)
    assert r["match"] == 2 and r["lower"] == 1 and r["higher"] == 1
    assert abs(r["max_abs_diff_matched"] - 5e-9) < 1e-15


def test_traffic_lookup_requires_matching_sources(tmp_path, monkeypatch):
    f = tmp_path / "t.json"
    entry = dict(kernel="eig", batch=256, source_sha256=bench.kernel_source_digest(),
                 fetch_kib_per_dispatch=10.0, write_kib_per_dispatch=100.0, fetch_scale=2.0, write_scale=1.0)
    f.write_text(json.dumps(entry))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("eig", 256) == 1024.0 * (10.0 * 2.0 + 100.0)
    assert bench.measured_traffic("eig", 64) is None
    assert bench.measured_traffic("forward", 256) is None
    entry["source_sha256"] = "0" * 64
    f.write_text(json.dumps(entry))
    assert bench.measured_traffic("eig", 256) is None
    monkeypatch.setattr(bench, "TRAFFIC_FILE", os.path.join(str(tmp_path), "missing.json"))
    assert bench.measured_traffic("eig", 256) is None


def test_algorithmic_flop_counts():
    n, p = 36, 32
    assert bench.alg_flops_per_step("eig", n, p) == 13 * n ** 3
    assert bench.alg_flops_per_step("forward", n, p) == 8 * n * n * p
    assert bench.alg_flops_per_step("sterm", n, p) == 8 * n ** 3
    # C2 per evaluation: J (21 N^3 + 16 N^2 P)
    f_alg = sum(bench.alg_flops_per_step(k, n, p) for k in ("eig", "forward", "backward", "sterm")) * 4000
    assert f_alg == 4000 * (21 * n ** 3 + 16 * n * n * p)
