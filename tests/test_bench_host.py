"""Host-side logic of the benchmark and the batch workload recipe (CPU)."""
import os

import numpy as np
import pytest

import bench
import synth


def test_recorded_traffic_is_tied_to_the_kernel_sources():
    """The committed counter summary holds for the kernel sources it was
    taken on: its bytes are reported while the source hash matches, and no
    figure is reported for a kernel it does not list."""
    path = os.path.join(bench.ROOT, "profiles", "hbm_traffic_slab96_q1.txt")
    lines = [ln for ln in open(path) if ln.strip().startswith("traffic ")]
    assert lines, "no machine-readable traffic lines"
    recorded = {}
    for ln in lines:
        _, kernel, b, src = ln.split()
        recorded[kernel] = (int(b.split("=")[1]), src.split("=")[1])
    for kernel, (nbytes, src) in recorded.items():
        got = bench.recorded_traffic("slab96_q1", kernel)
        assert got == (nbytes if src == bench.source_hash() else None), kernel
    assert bench.recorded_traffic("slab96_q1", "no_such_kernel") is None
    assert bench.recorded_traffic("no_such_workload", "apply_blocks_kernel<float,7>") is None


def test_recorded_valu_is_tied_to_the_kernel_sources():
    """The committed VALU counter summary likewise: instructions and
    wavefronts per launch while the source hash matches, else nothing; the
    bench's view derives the full-issue time from them."""
    path = os.path.join(bench.ROOT, "profiles", "valu_slab96_q1.txt")
    lines = [ln for ln in open(path) if ln.strip().startswith("valu ")]
    assert lines, "no machine-readable VALU lines"
    for ln in lines:
        _, kernel, ins, waves, src = ln.split()
        want = (int(ins.split("=")[1]), int(waves.split("=")[1]))
        got = bench.recorded_valu("slab96_q1", kernel)
        assert got == (want if src.split("=")[1] == bench.source_hash() else None), kernel
        if got is not None:
            view = bench.valu_view("slab96_q1", kernel, 1.0)
            assert abs(view["ms_at_full_issue"] - want[0] / (256 * 4 * 2.4e9 / 4) * 1e3) < 1e-3


def _profiles_current():
    stats = open(os.path.join(bench.ROOT, "profiles", "kernel_stats_slab96_q1.md")).read()
    return f"library source hash: {bench.source_hash()}" in stats


def test_committed_profiles_agree_with_each_other():
    """Both summaries were taken on the same kernel sources; when those are
    the current ones the benchmark's roofline carries measured traffic."""
    if not _profiles_current():
        pytest.skip("profiles taken on other kernel sources")
    assert bench.recorded_traffic("slab96_q1", "apply_blocks_bf16_kernel<7>") is not None
    assert bench.recorded_traffic("slab96_q1", bench.JVP_KERNEL["f32"]) is not None
    assert bench.recorded_valu("slab96_q1", bench.JVP_KERNEL["f32"]) is not None


def test_recorded_bytes_match_the_algorithmic_bytes_of_the_block_apply():
    """Counter-measured HBM bytes of the block applies agree with their
    algorithmic bytes (no wasted re-reads) to within 0.1 %."""
    if not _profiles_current():
        pytest.skip("profiles taken on other kernel sources")
    w = synth.WORKLOADS["slab96_q1"]
    ne = w.nx * w.ny * w.nz
    alg = {"apply_blocks_kernel<float,7>": ne * (56 * 56 + 2 * 56) * 4,
           "apply_blocks_bf16_kernel<7>": ne * (56 * 56 * 2 + 2 * 56 * 4)}
    for kernel, nbytes in alg.items():
        got = bench.recorded_traffic("slab96_q1", kernel)
        assert got is not None and abs(got / nbytes - 1.0) < 1e-3, (kernel, got, nbytes)


def test_batch_workload_recipe():
    """64 cubes with edges in 24..64 and porosities in [0.4, 0.75), mask
    seeds 1000 + b; the same seed gives the same batch."""
    specs = synth.batch_structures(64)
    assert len(specs) == 64
    edges = np.array([e for e, _, _ in specs])
    por = np.array([p for _, p, _ in specs])
    assert edges.min() >= 24 and edges.max() <= 64 and len(set(edges)) > 10
    assert por.min() >= 0.4 and por.max() < 0.75
    assert [m for _, _, m in specs] == [1000 + b for b in range(64)]
    assert synth.batch_structures(64) == specs


def test_bench_refuses_several_gpus(capsys):
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU" in capsys.readouterr().err
