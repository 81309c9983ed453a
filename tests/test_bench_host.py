"""CPU checks of bench.py's host-side accounting: which timed CG sweep-B
launches count as full sweeps for the roofline, and the counter-traffic
weighting of the sweep's two forms."""
import json
import os

import bench


def test_full_sweeps_from_iteration_tags():
    n, N = 10, 4
    blk = n * N * 8
    # step 1: 3 working iterations (tags 0, 1, 2) and one launch past
    # convergence (tag 3); step 2: 2 working (0, 1) and two past (2, 3)
    tags = [0, 1, 2, 3, 0, 1, 2, 3]
    ms = [1.0, 2.0, 1.5, 0.01, 1.1, 2.1, 0.02, 0.9]
    full, full_ms, full_bytes, parity = bench.full_sweep_b(tags, ms, [3, 2], len(tags), n, N)
    assert full == 5 and parity == [3, 2]
    assert abs(full_ms - (1.0 + 2.0 + 1.5 + 1.1 + 2.1)) < 1e-12
    assert full_bytes == 3 * (3 * blk + 8 * n) + 2 * (6 * blk + 8 * n)


def test_full_sweeps_need_tags_for_every_launch_and_step():
    # fewer tags than launches (a capped record) or a step count that does not
    # match the tag runs: no full sweeps reported
    assert bench.full_sweep_b([0, 1], [1.0, 1.0], [2], 3, 10, 4)[0] == 0
    assert bench.full_sweep_b([0, 1, 0], [1.0, 1.0, 1.0], [2], 3, 10, 4)[0] == 0
    # a step without any working iteration contributes nothing
    assert bench.full_sweep_b([0, 0, 1], [1.0, 1.0, 1.0], [0, 2], 3, 10, 4)[:2] == (2, 2.0)


def test_traffic_weighted_by_the_forms(tmp_path, monkeypatch):
    src = os.path.join(bench.ROOT, "paper_2511_06788_amd", "csrc", bench.PMC_SOURCES["cg_sweep_b"])
    import hashlib
    rec = {"n": 10, "N": 4, "copy_scale": 1.0, "fetch_kib_per_dispatch": 3.0, "write_kib_per_dispatch": 1.0,
           "per_kernel": [{"fetch_kib": 2.0, "write_kib": 1.0}, {"fetch_kib": 4.0, "write_kib": 2.0}],
           "source_sha256": hashlib.sha256(open(src, "rb").read()).hexdigest()}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "pmc_traffic_cg_sweep_b.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    # the source is looked up under ROOT: give the temporary root the same file
    d = tmp_path / "paper_2511_06788_amd" / "csrc"
    d.mkdir(parents=True)
    (d / bench.PMC_SOURCES["cg_sweep_b"]).write_bytes(open(src, "rb").read())
    assert bench.traffic_from_pmc(10, 4) == 4.0 * 1024
    assert bench.traffic_from_pmc(10, 4, mix=[3, 1]) == (3 * 3.0 + 1 * 6.0) / 4 * 1024
    assert bench.traffic_from_pmc(10, 5) is None                  # another workload
    (d / bench.PMC_SOURCES["cg_sweep_b"]).write_bytes(b"changed")
    assert bench.traffic_from_pmc(10, 4) is None                  # the kernel changed since the counters


def test_mixed_floor_rule():
    """The mixed phase of the long run ends once `chunk` steps lower the
    residual by less than 1%, and not before `chunk` steps have run."""
    chunk = 1500
    # a slow but steady phase: 10% per 1500 steps is not the floor
    steady = [(k * 100, 1e-3 * 0.9 ** (k / 15)) for k in range(40)]
    assert not bench.mixed_floor_reached(steady, chunk)
    # fewer steps than one chunk: no decision yet, however flat
    assert not bench.mixed_floor_reached([(0, 1e-4), (60, 1e-4), (120, 1e-4)], chunk)
    # flat over the last chunk: the floor
    flat = steady + [(4000 + k * 100, steady[-1][1] * (1 - 1e-4 * k)) for k in range(1, 20)]
    assert bench.mixed_floor_reached(flat, chunk)
    # a residual that rises again is at the floor too
    assert bench.mixed_floor_reached([(0, 1e-4), (1600, 1.2e-4)], chunk)
