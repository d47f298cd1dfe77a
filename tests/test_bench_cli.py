"""bench.py measures one GPU: any other --gpus value is refused before anything is loaded."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout == ""


def _bench():
    import importlib.util
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_code_hash_ignores_comments_but_not_code(tmp_path):
    b = _bench()
    a = tmp_path / "a.hip"
    a.write_text("int f(int x) {\n  return x + 1;\n}\n")
    h0 = b.code_hash(str(a))
    a.write_text("// header\nint f(int x) {  // trailing\n\n  return x + 1;\n}\n")
    assert b.code_hash(str(a)) == h0
    a.write_text("int f(int x) {\n  return x + 2;\n}\n")
    assert b.code_hash(str(a)) != h0


def test_traffic_is_reported_only_for_the_measured_sources():
    # the HBM traffic of a committed summary is reported while the kernel's sources hash to the
    # value recorded there, and only for the benchmark workload
    import stmg_inputs as si
    b = _bench()
    cfg = si.paper_config(2)
    for key in ("operator", "smoother"):
        path, src = b.TRAFFIC_PROFILES[key]
        rec = {}
        for line in open(path):
            if ":" in line:
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        cur = b.code_hash(*[os.path.join(ROOT, "paper_2408_04372_amd", "csrc", f) for f in src])
        t = b.kernel_traffic(cfg, key)
        if rec.get("source_sha256_16") == cur:
            assert t == float(rec["traffic_bytes_per_apply"]), key
        else:
            assert t is None, key
        assert b.kernel_traffic(si.paper_config(3), key) is None
