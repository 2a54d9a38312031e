"""Host-side parts of bench.py: the one-GPU refusal and the reading of the
committed rocprofv3 summaries (values are reported only for the kernel source
they were measured on)."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_profile_values_follow_the_kernel_source(tmp_path, monkeypatch):
    b = _bench_module()
    prof = tmp_path / "profiles"
    prof.mkdir()
    sha = b._kernel_source_sha()
    (prof / "x.txt").write_text("# comment: 1\nevaluate_hip_sha256_16: %s\nm2l_mfma_busy_bf16x3: 0.5   (note)\n" % sha)
    (prof / "y.txt").write_text("evaluate_hip_sha256_16: 0000000000000000\nm2l_mfma_busy_bf16x3: 0.5\n")
    # the summaries are looked up under ROOT/profiles; the kernel source stays the real one
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setattr(b, "_kernel_source_sha", lambda: sha)
    assert b._profile_value("x.txt", "m2l_mfma_busy_bf16x3") == 0.5
    assert b._profile_value("x.txt", "missing_key") is None
    assert b._profile_value("y.txt", "m2l_mfma_busy_bf16x3") is None  # another kernel source
    assert b._profile_value("absent.txt", "m2l_mfma_busy_bf16x3") is None


def test_committed_summaries_parse():
    b = _bench_module()
    for name, key in (("m2l_traffic_uniform1m_p6.txt", "traffic_bytes_bf16x3"),
                      ("m2l_mfma_util_uniform1m_p6.txt", "m2l_mfma_busy_bf16x3")):
        path = os.path.join(ROOT, "profiles", name)
        assert os.path.exists(path), name
        kv = {}
        for line in open(path):
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
        assert "evaluate_hip_sha256_16" in kv and key in kv, name
        if kv["evaluate_hip_sha256_16"] == b._kernel_source_sha():
            assert b._profile_value(name, key) is not None
