"""CPU tests of the host price loop (L-BFGS / subgradient state machine)
against fake evaluators with known minimisers (tests/price_loop_harness.cpp)."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def harness(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("pl") / "price_loop_harness")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-I", os.path.join(ROOT, "include"),
                           "-I", os.path.join(ROOT, "paper_2104_00282_amd", "csrc"),
                           os.path.join(ROOT, "tests", "price_loop_harness.cpp"), "-o", exe])
    return exe


def run(exe, mode):
    out = subprocess.check_output([exe, mode], text=True).split()
    d = {}
    for kv in out:
        k, v = kv.split("=")
        d[k] = float(v)
    return d


def test_interior_minimiser(harness):
    d = run(harness, "interior")
    assert d["converged"] == 1 and d["err"] < 1e-5
    assert d["iters"] < 40 and d["fallbacks"] == 0


def test_boundary_minimiser_projected(harness):
    d = run(harness, "boundary")
    assert d["converged"] == 1 and d["err"] < 1e-5


def test_subgradient_method(harness):
    d = run(harness, "subgradient")
    assert d["fallbacks"] == d["iters"] > 0
    assert d["err"] < 0.5


def test_eval_budget_is_exact(harness):
    d = run(harness, "budget")
    assert d["evals"] == 7 and d["calls"] == 7 and d["converged"] == 0


def test_stall_stop(harness):
    d = run(harness, "stall")
    assert d["stalled"] == 1 and d["converged"] == 0 and d["evals"] < 200


def test_stall_restarts(harness):
    """With stall_restarts = 3 the first three stalls restart the update from
    the best certified point (empty memory: a projected steepest-descent step
    of the default length), and the fourth stops the loop."""
    base = run(harness, "stall")
    d = run(harness, "stall_restart")
    assert base["restarts"] == 0
    assert d["restarts"] == 3 and d["restart_checks"] == 3 and d["restart_ok"] == 1
    assert d["stalled"] == 1 and d["converged"] == 0
    assert d["evals"] > base["evals"] + 3 * 25 - 1
    assert d["rel"] <= base["rel"]


def test_inconsistent_gradient_falls_back(harness):
    d = run(harness, "badgrad")
    assert d["done"] == 1 and d["fallbacks"] > 0
