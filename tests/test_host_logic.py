"""Host-side behaviour that needs no GPU: the bench's one-GPU contract and busy-span arithmetic, the
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


def test_bench_busy_span_is_the_union_of_launch_intervals():
    sys.path.insert(0, ROOT)
    import bench
    assert bench.union_ms([]) == 0.0
    assert bench.union_ms([(0.0, 2.0)]) == 2.0
    # overlapping, nested, touching and disjoint intervals, in any order
    assert bench.union_ms([(5.0, 6.0), (0.0, 2.0), (1.0, 3.0), (1.5, 1.8), (3.0, 4.0)]) == 5.0
    assert bench.union_ms([(0.0, 10.0), (2.0, 3.0), (9.0, 12.0), (20.0, 21.0)]) == 13.0


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
