"""Host-side behaviour that needs no GPU: the bench's one-GPU contract, its iteration table and traffic gate, the
relative-binning edge function's argument handling, and argument checks of the sampler entry points (rejected
before any device call)."""
import ctypes
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_bench_queue_model_and_start_order():
    """The queue model behind the bench's tail figures: slots take particles in order and share their compute
    unit (the leaf time grows from lone_us with one busy slot to full_us with every slot busy); a bad order leaves
    slots idle in the tail, longest first does not; the start order is the launch's log2 buckets of the hint,
    descending and stable."""
    sys.path.insert(0, ROOT)
    import bench
    span, occ = bench.queue_span([3, 2], [0, 1], 1, 1.0, 1.0)
    assert span == pytest.approx(5.0) and occ == pytest.approx(1.0)
    span, occ = bench.queue_span([4, 4, 4, 4], [0, 1, 2, 3], 2, 1.0, 1.0)
    assert span == pytest.approx(8.0) and occ == pytest.approx(1.0)
    span, occ = bench.queue_span([1, 1, 1, 3], [0, 1, 2, 3], 2, 1.0, 1.0)
    assert span == pytest.approx(4.0) and occ == pytest.approx(0.75)
    span, occ = bench.queue_span([1, 1, 1, 3], [3, 0, 1, 2], 2, 1.0, 1.0)
    assert span == pytest.approx(3.0) and occ == pytest.approx(1.0)
    # contention: two busy slots take the full-load leaf time, a lone one the lone time
    assert bench.queue_span([1, 1], [0, 1], 2, 1.0, 2.0)[0] == pytest.approx(2.0)
    assert bench.queue_span([1], [0], 2, 1.0, 2.0)[0] == pytest.approx(1.0)
    # particles without leaves take no slot time
    assert bench.queue_span([0, 2, 0], [0, 1, 2], 1, 1.0, 1.0)[0] == pytest.approx(2.0)
    assert bench.start_order([0, 5, 100, 5, 1]).tolist() == [2, 1, 3, 4, 0]
    # without a hint: stripes of 16 neighbours dealt to 8 queues, the queues taken side by side
    order = bench.striped_order(300)
    assert sorted(order.tolist()) == list(range(300))
    assert order[:3].tolist() == [0, 16, 32] and order[8:10].tolist() == [1, 17]
    assert order[127] == 127 and order[128] == 128 and order[256:259].tolist() == [256, 272, 288]


def test_bench_busy_time_is_the_union_of_launch_intervals():
    """Launches on several streams overlap: the kernel's busy time is the length of the union of their
    intervals (nested, touching, disjoint and unsorted intervals; one stream's back-to-back launches give their
    summed durations)."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.union_ms([], []) == 0.0
    assert bench.union_ms([5.0, 0.0, 1.0], [6.0, 2.0, 3.0]) == pytest.approx(4.0)
    assert bench.union_ms([0.0, 0.5], [3.0, 1.0]) == pytest.approx(3.0)
    assert bench.union_ms([0.0, 2.0], [2.0, 4.0]) == pytest.approx(4.0)
    s = [0.0, 10.0, 25.0]
    e = [9.0, 20.0, 26.0]
    assert bench.union_ms(s, e) == pytest.approx(sum(b - a for a, b in zip(s, e)))


def test_bench_iteration_table_and_traffic_gate(tmp_path, monkeypatch):
    """The per-iteration rows are the runs' records divided by the run size (the largest divergent fraction over
    the runs), and counter traffic is reported only for the kernel sources, kernel and command it was taken on
    (the first of the committed summaries that matches all three)."""
    sys.path.insert(0, ROOT)
    import bench
    from paper_2601_02336_amd import smcgw
    h = np.zeros((2, 3, smcgw.HIST_SIZE))
    h[:, :, smcgw.H_BETA] = [[0.1, 0.2, 0.3], [0.15, 0.25, 0.35]]
    h[:, :, smcgw.H_DIVERGENT] = [[1, 0, 5], [2, 0, 1]]
    h[:, :, smcgw.H_DEPTH] = [[40, 60, 80], [40, 60, 100]]
    h[:, :, smcgw.H_LEAPFROG] = [[100, 200, 300], [1, 2, 3]]
    rows = bench.iteration_table(smcgw, h, 20)
    assert [r["divergent_frac"] for r in rows] == [0.1, 0.0, 0.25]
    assert [r["mean_depth"] for r in rows] == [2.0, 3.0, 4.5]
    assert [r["leapfrog"] for r in rows] == [101, 202, 303]
    assert rows[2]["beta"] == [0.3, 0.35]
    f = tmp_path / "traffic.txt"
    g = tmp_path / "traffic_other_layout.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILES", [str(tmp_path / "absent.txt"), str(g), str(f)])
    assert bench.measured_traffic("k", "") is None                       # no file
    g.write_text("kernel=k\nbench_args=--steps 3 --layout streams\nsource_sha256={}\ntraffic_bytes_per_launch=9\n"
                 "fetch_bytes_per_launch=6\nwrite_bytes_per_launch=3\n".format(bench.kernel_source_hash()))
    assert bench.measured_traffic("k", "--steps 3 --layout streams")["bytes_per_launch"] == 9
    body = ("# made by a counter run\nkernel=k\nbench_args=--steps 3\nsource_sha256={}\n"
            "traffic_bytes_per_launch=30\nfetch_bytes_per_launch=20\nwrite_bytes_per_launch=10\n")
    f.write_text(body.format(bench.kernel_source_hash()))
    assert bench.measured_traffic("k", "--steps 3") == {"bytes_per_launch": 30, "fetch_bytes_per_launch": 20,
                                                        "write_bytes_per_launch": 10}
    assert bench.measured_traffic("other", "--steps 3") is None          # another kernel
    assert bench.measured_traffic("k", "") is None                       # another command
    f.write_text(body.format("0" * 64))
    assert bench.measured_traffic("k", "--steps 3") is None              # other sources


def test_rb_edges_arguments():
    from paper_2601_02336_amd import smcgw
    L = smcgw.lib()
    out = np.zeros(8, dtype=np.int32)
    p = out.ctypes.data_as(ctypes.c_void_p)
    assert L.smcgw_rb_edges(20.0, 0.5, 1, 0.1, p, 8) == smcgw.ERR_INVALID        # a single bin
    assert L.smcgw_rb_edges(20.0, 0.0, 100, 0.1, p, 8) == smcgw.ERR_INVALID      # df = 0
    assert L.smcgw_rb_edges(0.0, 0.5, 100, 0.1, p, 8) == smcgw.ERR_INVALID       # f_low = 0
    assert L.smcgw_rb_edges(20.0, 0.5, 100, 0.0, p, 8) == smcgw.ERR_INVALID      # eps = 0
    assert L.smcgw_rb_edges(20.0, 0.5, 1000, 0.01, p, 8) == smcgw.ERR_SHAPE      # more edges than room
    # two bins: the edges are the two ends
    assert L.smcgw_rb_edges(20.0, 0.5, 2, 0.1, p, 8) == 2 and list(out[:2]) == [0, 1]
    # a huge tolerance: one bin over the whole band
    e = smcgw.rb_edges(20.0, 0.25, 1969, 1e6)
    assert list(e) == [0, 1968]


def test_sampler_entry_points_reject_bad_arguments():
    from paper_2601_02336_amd import smcgw
    L = smcgw.lib()
    d, u = ctypes.c_double, ctypes.c_uint64
    # NULL context or arrays, alpha outside (0, 1], NULL output buffer
    assert L.smcgw_smc_reweight_resample_async(None, 4, 1, d(0.0), d(0.5), u(0), u(0), None, None, None, None,
                                               None, None) == smcgw.ERR_INVALID
    assert L.smcgw_ps_reweight_resample(None, 2, 4, 1, None, None, None, None, None, d(1.5), u(0), u(0), None, None,
                                        None, None, None, None) == smcgw.ERR_INVALID
    assert L.smcgw_recycle(None, 0, 4, None, None, None, u(0), None, None, None, None) == smcgw.ERR_INVALID
    assert L.smcgw_add_event_rb(None, None, None, None, None, None, d(0.1), None, None) == smcgw.ERR_INVALID


def test_iteration_entry_points_reject_bad_arguments():
    """The whole-iteration call, its graph and the plain comparison form refuse NULL contexts, descriptors and
    handles before any device call."""
    from paper_2601_02336_amd import smcgw
    L = smcgw.lib()
    desc = smcgw.SmcIterDesc()
    assert L.smcgw_smc_iteration(None, None) == smcgw.ERR_INVALID
    assert L.smcgw_smc_iteration(None, ctypes.byref(desc)) == smcgw.ERR_INVALID
    out = ctypes.c_void_p()
    assert L.smcgw_smc_graph_create(None, ctypes.byref(desc), ctypes.byref(out)) == smcgw.ERR_INVALID
    assert L.smcgw_smc_graph_create(None, ctypes.byref(desc), None) == smcgw.ERR_INVALID
    assert L.smcgw_graph_launch(None, 1) == smcgw.ERR_INVALID
    assert L.smcgw_graph_destroy(None) == smcgw.ERR_INVALID
    assert L.smcgw_loglike_grad_tangent(None, 4, None, None, None, None) == smcgw.ERR_INVALID
    assert L.smcgw_loglike_grad_noalloc(None, 4, None, None, None, None, smcgw.MIXED) == smcgw.ERR_INVALID
