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
    # value recorded there, and only for the workload it was measured on
    import stmg_inputs as si
    b = _bench()
    by_name = {si.paper_config(i).name: si.paper_config(i) for i in range(1, 6)}
    for (name, key), (fname, src) in b.TRAFFIC_PROFILES.items():
        cfg = by_name[name]
        path = os.path.join(ROOT, "profiles", fname)
        t = b.kernel_traffic(cfg, key)
        if not os.path.exists(path):
            assert t is None, (name, key)
            continue
        rec = {}
        for line in open(path):
            if ":" in line:
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
        cur = b.code_hash(*[os.path.join(ROOT, "paper_2408_04372_amd", "csrc", f) for f in src])
        if rec.get("source_sha256_16") == cur and rec.get("dtype", "f64") == "f64":
            assert t == float(rec["traffic_bytes_per_apply"]), (name, key)
        else:
            assert t is None, (name, key)
    # no summary covers the wave workload
    assert b.kernel_traffic(si.paper_config(3), "operator") is None
    assert b.kernel_traffic(si.paper_config(3), "smoother") is None
