"""Host-side checks of bench.py's arithmetic (no GPU): the roofline terms
against the worked figures of the traversal's byte and operation model,
the guard on the committed traffic counters, the U-Net's FLOP count on
small networks counted by hand, and the one-GPU contract of --gpus."""
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_roofline_bytes_match_the_worked_example():
    """20 node visits and 24 triangle tests per closest-hit ray cost
    32 + 16 + 20 * 256 + 24 * 36 = 6032 bytes (about 6.0 KB); 0.66 G such
    rays per second then move about half of the 8 TB/s peak."""
    n = 660_000_000
    r = bench._kernel_roofline("k", "k<false>", 1, 1000.0, n, 0, 20 * n, 24 * n, 1, "large")
    assert r["alg_bytes_per_launch"] == 6032 * n
    assert r["achieved"] == pytest.approx(6032 * 0.66, abs=0.05)   # reported to 0.1 GB/s
    assert 0.49 < r["frac"] < 0.51
    assert r["nodes_per_ray"] == 20 and r["tris_per_ray"] == 24


def test_roofline_operations_match_the_worked_example():
    """14 operations per child box of an 8-wide node and 40 per triangle:
    20 nodes and 24 triangles are 3200 operations, so 39.3 T lane
    operations per second bound the kernel at about 12.3 G rays per
    second."""
    n = int(256 * 64 * 2.4e9 / 3200)   # rays per second at the VALU peak
    r = bench._kernel_roofline("k", "k<false>", 1, 1000.0, n, 0, 20 * n, 24 * n, 1, "large")
    assert r["valu"]["ops_per_launch"] == 3200 * n
    assert r["valu"]["frac"] == pytest.approx(1.0, rel=1e-3)
    assert 12.2e3 < r["kernel_Mrays_s"] < 12.4e3


def test_roofline_shadow_rays_and_launch_averages():
    """Shadow rays write 4 bytes of occlusion instead of a 16-byte hit;
    figures are per launch, time per step divides by the steps."""
    r = bench._kernel_roofline("k", "k<false>", 4, 40.0, 0, 1000, 0, 0, 2, "medium")
    assert r["alg_bytes_per_launch"] == round(1000 * 36 / 4)
    assert r["avg_launch_ms"] == 10.0
    assert r["ms_per_step"] == 20.0
    assert bench._kernel_roofline("k", "k<false>", 0, 0.0, 1, 0, 0, 0, 1, "large") is None


def test_traffic_counters_only_for_the_sources_they_were_taken_on(monkeypatch):
    """The committed counter summary carries the hash of the traversal
    sources it was taken on; a different hash, or a kernel it does not
    list, gives no traffic figure."""
    path = bench.TRAFFIC_FILES["large"]
    txt = open(path).read()
    line = [ln for ln in txt.splitlines() if ln.startswith("hbm_bytes_per_launch k_finish_camera<false, false>:")]
    assert line, "the large-scene summary lists the camera finishing kernel"
    listed = float(line[0].split(":")[1])
    stamp = [ln for ln in txt.splitlines() if ln.startswith("source_hash:")][0].split(":")[1].strip()
    monkeypatch.setattr(bench, "_src_hash", lambda: stamp)
    assert bench._traffic_per_launch("k_finish_camera<false, false>", "large") == listed
    assert bench._traffic_per_launch("k_no_such_kernel<false>", "large") is None
    monkeypatch.setattr(bench, "_src_hash", lambda: "0" * 16)
    assert bench._traffic_per_launch("k_finish_camera<false, false>", "large") is None


def test_unet_flops_counted_by_hand():
    """One level: two 3x3 convolutions (in -> c, c -> c) and the 1x1 output
    layer.  Two levels: the same at full and quarter size, then the
    decoder's 3x3 convolution of the upsampled deep features concatenated
    with the skip ((b + a) -> a), its second convolution (a -> a) and the
    output layer, at full size."""
    h, w, i, o = 16, 24, 9, 3
    a, b = 8, 12
    one = 2 * h * w * 9 * (i * a + a * a) + 2 * h * w * a * o
    assert bench.unet_flops([a], h, w, i, o) == one
    enc = 2 * h * w * 9 * (i * a + a * a) + 2 * (h // 2) * (w // 2) * 9 * (a * b + b * b)
    dec = 2 * h * w * 9 * ((b + a) * a + a * a)
    assert bench.unet_flops([a, b], h, w, i, o) == enc + dec + 2 * h * w * a * o


def test_more_than_one_gpu_is_refused():
    """The benchmark runs on one GPU; asked for more it exits with status 2
    and says so, before it touches a GPU."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stdout
