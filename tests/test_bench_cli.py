"""What of bench.py needs no GPU: more than one GPU is refused with a JSON
error line and exit status 2, and the committed profiles it reads are those
of the current kernel sources."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    line = json.loads(p.stdout.strip().splitlines()[-1])
    assert "one GPU" in line["error"]


def test_committed_profiles_match_the_kernel_sources():
    """The counter summaries the bench line reads (traffic, VALU issue) and
    the kernel-trace statistics were all taken on the kernel sources as they
    stand; an edit to a kernel without a new profile fails here, rather than
    silently turning the bench line's traffic into null."""
    sys.path.insert(0, ROOT)
    import bench
    sha, sha_m = bench.source_sha("resampling"), bench.source_sha("mlp")
    for what in ("traffic", "sq_counters"):
        with open(os.path.join(ROOT, "profiles", f"k_initial_hd_{what}.json")) as fh:
            assert json.load(fh)["source_sha"] == sha, what
    with open(os.path.join(ROOT, "profiles", "k_reuse_hd_sq_counters.json")) as fh:
        reuse = json.load(fh)
    assert reuse["kernel_sources"] == sha
    assert set(reuse["kernels"]) == set(bench.REUSE_KERNELS)
    for name, h in (("k_initial_hd_kernel_stats.txt", sha), ("k_mlp_infer_hd_kernel_stats.txt", sha_m),
                    ("k_mlp_infer_hd_mfma_counters.txt", sha_m)):
        with open(os.path.join(ROOT, "profiles", name)) as fh:
            assert f"kernel sources: {h}" in fh.read(), name
    # the bench line's algorithmic bytes: 104 B per pixel of the 1920x1080 frame
    assert bench.measured_traffic("k_initial", "hd") > 104 * 1920 * 1080
    issue = bench.alu_issue("k_initial", "hd", 6.0)
    assert issue is not None and 0.0 < issue["frac"] < 1.0
