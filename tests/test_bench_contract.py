"""Host-side checks of the benchmark script's contract (no GPU).

* More than one GPU is refused with a message (the shot-parallel multi-GPU
  layout is described, not built) before anything touches a device.
* The committed counter profiles carry the machine-readable values the
  benchmark reads, and the algorithmic bytes it reports per kernel never
  exceed what the counters measured for that kernel (the byte model counts
  every array once; the counters add halo re-reads, partial lines and the
  absorbing strips), and were taken on the kernel sources in the tree.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def _profile_values(tag):
    vals = {}
    for line in open(os.path.join(ROOT, "profiles", f"pmc_{tag}.md")):
        line = line.strip()
        if line.startswith("- ") and ":" in line:
            k, v = line[2:].split(":", 1)
            vals[k.strip()] = v.strip()
    return vals


@pytest.mark.parametrize("tag,ndim", [("config2_batched", 2), ("config5_batched", 3)])
def test_profiles_bound_the_byte_model(tag, ndim):
    import bench
    vals = _profile_values(tag)
    assert len(vals.get("kernel_source_sha", "")) == 16
    assert int(vals["points_per_launch"]) > 0
    for kernel, alg in bench.BYTES_PER_PT[ndim].items():
        measured = float(vals[f"traffic_bytes_per_point.{kernel}"])
        assert alg <= measured <= 2.0 * alg, (kernel, alg, measured)


@pytest.mark.parametrize("tag,ndim", [("config2_batched", 2), ("config5_batched", 3)])
def test_profiles_describe_the_committed_kernels(tag, ndim):
    """The committed counter profile was taken on the kernel sources in the
    tree (the benchmark reports its traffic only then): a kernel edit must
    come with a new profile."""
    import bench
    assert _profile_values(tag)["kernel_source_sha"] == bench.kernel_source_hash(ndim)
    assert bench.read_traffic(tag, "adj_a", 1.0, ndim) is not None
