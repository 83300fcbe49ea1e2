"""Host-side checks of the benchmark's accounting: the per-kernel split of the
algorithmic bytes, the HBM-traffic summary and the one-GPU guard."""
from __future__ import annotations

import csv
import json
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402

KINDS = ("k_predict", "k_epoch_empty", "k_traverse_queue")


def random_counters(g):
    """Counters of one HRPP call that respect the schedule's identities."""
    n = int(g.integers(1000, 100000))
    e_rays = int(g.integers(0, n))                 # rays of the first epoch after a reset
    e_inv = int(g.integers(0, max(1, e_rays // 10)))
    e_look = e_rays - e_inv
    inv = e_inv + int(g.integers(0, max(1, (n - e_rays) // 10)))
    lookups = n - inv
    pos = int(g.integers(0, lookups - e_look + 1))
    pred_hits = int(g.integers(0, pos + 1))
    fallback = lookups - e_look - pred_hits        # negatives and false positives traverse
    q_trav = int(g.integers(0, fallback + 1))
    traversals = e_look + fallback
    e_int, e_tri = int(g.integers(0, 40 * e_look + 1)), int(g.integers(0, 12 * e_look + 1))
    q_int, q_tri = int(g.integers(0, 40 * q_trav + 1)), int(g.integers(0, 12 * q_trav + 1))
    i_int, i_tri = int(g.integers(0, 40 * (fallback - q_trav) + 1)), int(g.integers(0, 12 * (fallback - q_trav) + 1))
    p_box, p_tri = int(g.integers(0, 8 * pos + 1)), int(g.integers(0, 32 * pos + 1))
    e_rec = int(g.integers(0, e_look + 1))
    q_rec = int(g.integers(0, q_trav + 1))
    i_rec = int(g.integers(0, fallback - q_trav + 1))
    return dict(rays=n, invalid=inv, lookups=lookups, pred_hits=pred_hits, traversals=traversals,
                interior_visited=e_int + q_int + i_int, tri_tests=e_tri + q_tri + i_tri + p_tri,
                pred_box_tests=p_box, pred_tri_tests=p_tri, records=e_rec + q_rec + i_rec,
                queue_traversals=q_trav, queue_interior_visited=q_int, queue_tri_tests=q_tri, queue_records=q_rec,
                empty_lookups=e_look, empty_rays=e_rays, empty_interior_visited=e_int, empty_tri_tests=e_tri,
                empty_records=e_rec)


def test_kernel_bytes_split_adds_up():
    # the prediction, first-epoch and queue kernels together move what the whole
    # call does: every ray once, a table entry per non-empty lookup, the predicted
    # leaves, one result per success or traversal, every traversal's nodes,
    # triangles and record, and the queue's entries (written, then read)
    g = np.random.default_rng(7)
    for _ in range(200):
        sa, sb = random_counters(g), random_counters(g)
        entry_b = int(g.choice([32, 64]))
        split = sum(bench.kernel_bytes(k, sa, sb, entry_b, sa["rays"], sb["rays"]) for k in KINDS)
        whole = 0
        for st, out_b in ((sa, 1), (sb, 16)):
            e_inv = st["empty_rays"] - st["empty_lookups"]
            whole += (st["rays"] * bench.RAY_B + (st["lookups"] - st["empty_lookups"]) * entry_b
                      + bench.LEAFBOX_B * st["pred_box_tests"] + bench.TRI_B * st["tri_tests"]
                      + (st["pred_hits"] + st["traversals"] + e_inv) * out_b
                      + bench.NODE_B * st["interior_visited"] + 20 * st["records"]
                      + st["queue_traversals"] * (8 + 8 + bench.RAY_B))
        assert split == whole


def test_kernel_ops_split_adds_up():
    # the prediction, first-epoch and queue kernels together do the call's
    # algorithmic VALU work: every ray's setup (a queued ray's again in the queue
    # kernel), the hash of every non-empty lookup and of every record, every box
    # test (root tests of the traversals, two per interior visit, the predicted
    # boxes) and every triangle test
    g = np.random.default_rng(8)
    for _ in range(200):
        sa, sb = random_counters(g), random_counters(g)
        split = sum(bench.kernel_ops(k, sa, sb) for k in KINDS)
        whole = 0
        for st in (sa, sb):
            whole += (bench.OPS_RAY * (st["rays"] + st["queue_traversals"])
                      + bench.OPS_HASH * (st["lookups"] - st["empty_lookups"] + st["records"])
                      + bench.OPS_BOX * (st["traversals"] + 2 * st["interior_visited"] + st["pred_box_tests"])
                      + bench.OPS_TRI * st["tri_tests"])
        assert split == whole


def test_stream_bytes_are_part_of_the_logical_bytes():
    # the streamed part (rays, results, queue and record writes) never exceeds the
    # kernel's logical bytes, and equals them when nothing is gathered
    g = np.random.default_rng(9)
    for _ in range(100):
        sa, sb = random_counters(g), random_counters(g)
        for k in KINDS + ("k_traverse_plain",):
            assert 0 <= bench.kernel_stream_bytes(k, sa, sb, 64, sa["rays"], sb["rays"]) <= bench.kernel_bytes(
                k, sa, sb, 64, sa["rays"], sb["rays"])
    st = {k: 0 for k in random_counters(np.random.default_rng(1))}
    st.update(rays=10)
    assert bench.kernel_stream_bytes("k_traverse_plain", st, st, 64, 10, 10) == bench.kernel_bytes(
        "k_traverse_plain", st, st, 64, 10, 10)


def test_valu_peak_from_unit_counts():
    # 256 CUs x 64 fp32 lanes per clock x 2.4 GHz, a quarter of the 157.3 TFLOP/s
    # vector peak (which counts an FMA as two flops and packed FP32 as two lanes)
    assert abs(bench.VALU_PEAK_TOPS - 39.3216) < 1e-3
    assert abs(4 * bench.VALU_PEAK_TOPS - 157.3) < 0.1


def test_kernel_bytes_plain_and_update():
    st = {k: 0 for k in random_counters(np.random.default_rng(1))}
    st.update(rays=10, interior_visited=7, tri_tests=3, records=5)
    assert bench.kernel_bytes("k_traverse_plain", st, st, 64, 10, 10) == (
        10 * (32 + 1) + 64 * 7 + 48 * 3 + 10 * (32 + 16) + 64 * 7 + 48 * 3)
    assert bench.kernel_bytes("k_update_apply", st, st, 64, 10, 10) == 2 * 5 * (24 + 64)


def test_traffic_summary_scales_by_the_copy_and_keeps_kernels_apart(tmp_path):
    # a copy of CALIB_BYTES that reads half its size as FETCH_SIZE scales fetch
    # bytes by 2; per-dispatch averages are kept per kernel, with the first-epoch
    # kernel apart from the prediction kernel
    def write(path, counter, rows):
        with open(path, "w", newline="") as fh:
            w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
            w.writeheader()
            for name, kib in rows:
                w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": kib})
    calib_kib = bench.CALIB_BYTES / 1024
    f = tmp_path / "f.csv"
    wcsv = tmp_path / "w.csv"
    write(f, "FETCH_SIZE", [("void at::native::elementwise_copy", calib_kib / 2),
                            ("void hrpp::k_predict<false, false, false, false, true>(...)", 100.0),
                            ("void hrpp::k_predict<true, false, false, false, true>(...)", 300.0),
                            ("void hrpp::k_epoch_empty<true, false, false>(...)", 1000.0)])
    write(wcsv, "WRITE_SIZE", [("void at::native::elementwise_copy", calib_kib),
                               ("void hrpp::k_predict<false, false, false, false, true>(...)", 10.0),
                               ("void hrpp::k_predict<true, false, false, false, true>(...)", 30.0),
                               ("void hrpp::k_epoch_empty<true, false, false>(...)", 7.0)])
    out = tmp_path / "t.json"
    bench.summarize_traffic(str(f), str(wcsv), str(out), configs=[{"x": 1}])
    d = json.load(open(out))
    assert d["fetch_scale"] == 2.0 and d["write_scale"] == 1.0
    kp, ke = d["kernels"]["k_predict"], d["kernels"]["k_epoch_empty"]
    assert kp["dispatches"] == 2 and kp["fetch_bytes_avg"] == 2.0 * 200.0 * 1024
    assert kp["write_bytes_avg"] == 20.0 * 1024
    assert ke["dispatches"] == 1 and ke["fetch_bytes_avg"] == 2.0 * 1000.0 * 1024


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
