"""Host-side checks of bench.py: the one-GPU guard, the lookup of the
committed HBM counters for the kernels its roofline names, the default
workload and the host baseline's sampling."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def load_bench():
    spec = importlib.util.spec_from_file_location("bench", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def _summaries(b):
    out = []
    for w in ("point512", "large2048"):
        path = b.PROFILE_JSON.format(workload=w)
        if os.path.exists(path):
            out.append((w, json.load(open(path))))
    return out


def test_profiled_names_exist_in_counter_summary():
    b = load_bench()
    found = _summaries(b)
    assert found
    for _, z in found:
        # the dominant kernel and the splat of the precision that was profiled
        assert b.PROFILED_NAME["k_rk4"] in z["kernels"]
        assert any(b.PROFILED_NAME[k] in z["kernels"]
                   for k in ("k_splat_binned", "k_splat_binned_split"))
        for kern in b.KERNEL_SOURCES:
            if b.PROFILED_NAME[kern] in z["kernels"]:
                assert kern in z["source_sha"], kern


def test_traffic_follows_source_hash(tmp_path, monkeypatch):
    b = load_bench()
    for w, z in _summaries(b):
        # with the stored hash replaced, the traffic must be withheld
        z["source_sha"] = {k: "0" * 16 for k in z["source_sha"]}
        (tmp_path / f"{w}_hbm_counters.json").write_text(json.dumps(z))
        monkeypatch.setattr(b, "PROFILE_JSON", str(tmp_path / "{workload}_hbm_counters.json"))
        for kern in b.KERNEL_SOURCES:
            assert b.profiled_traffic(kern, w) is None


def test_default_headline_is_the_largest_configuration():
    b = load_bench()
    sys_argv = sys.argv
    try:
        sys.argv = ["bench.py"]
        args = b.parse()
    finally:
        sys.argv = sys_argv
    assert args.workload == "large2048" and args.steps >= 5 and args.graph_steps >= 1


def test_cpu_baseline_on_a_small_workload():
    """The host baseline samples the FBI windows and the beams it says it
    does and scales them to the job: on the 128 x 128 wave-packet workload
    (the oracle finishes the sample in seconds) the figures are positive,
    the stage estimates add up to the job time, and the sample text names
    the counts."""
    import fga_inputs as fi
    b = load_bench()
    W = fi.workload("wavepacket", "fp64")
    nb = 1_000_000
    r = b.cpu_baseline(W, nb, 2.0)
    est = r["est_seconds"]
    assert set(est) == {"fbi", "rk4", "reconstruct"} and min(est.values()) > 0
    assert abs(nb / sum(est.values()) - r["value"]) <= 1e-9 * r["value"]
    assert r["kind"] == "oracle" and r["unit"] == "beams/s" and r["cores"] >= 1
    assert "10240 beams" in r["sample"] and "of 4096 q nodes" in r["sample"]
