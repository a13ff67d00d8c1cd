"""Pins of the oracle's convergence bookkeeping.  The paper relaxes to fixed physical end times and
defines no residual, so the build reads one in (a windowed kinetic-energy ratio):

    E_k(n)    = 1/2 sum over free particles of m |v_i|^2 after step n
    E_peak(n) = the largest E_k since the last reset of the tracking
    r_n       = max of E_k over the last W steps since that reset, divided by E_peak(n)
                (1 while E_peak = 0)
    stop      = the first step with r_n < tol and step index >= W

Everything here is recomputed from the oracle's own velocities, read back one step at a time, with
an exactly rounded sum, and must agree with what the oracle reports.  Three mistakes planted in a
copy of the oracle -- the current E_k in place of the window maximum, the n >= W condition dropped,
E_peak not raised when E_k grows -- must each fail the same checks.
"""
import math
import os
import subprocess

import numpy as np
import pytest

import oracle
import workloads

SEG1, SEG2 = 1300, 400          # steps before and after a reset of the tracking (set_state)
STOP_TOLS = (1.5, 0.1, 0.01)    # tol > 1: r_n <= 1 < tol always, so n >= W alone decides


def _body():
    return workloads.small_body(2, (20, 4), nclamp=2, alpha=0.5, jitter=0.05, jitter_seed=3)


def _ek(body, v):
    """1/2 sum_free m |v|^2: each particle's |v|^2 summed over components left to right, the
    particles' terms added with an exactly rounded sum."""
    D = body.dim
    vol = body.dp * body.dp * body.dp if D == 3 else body.dp * body.dp
    m = body.rho0 * vol
    vf = v[body.clamped == 0]
    vn2 = vf[:, 0] * vf[:, 0] + vf[:, 1] * vf[:, 1]
    if D == 3:
        vn2 = vn2 + vf[:, 2] * vf[:, 2]
    return math.fsum((0.5 * m) * vn2)


def _residuals(ek, W):
    """r_n for n = 1 .. len(ek) of one tracking segment (ek[0] is the first step after the reset)."""
    out = []
    peak = 0.0
    for n in range(1, len(ek) + 1):
        peak = max(peak, ek[n - 1])
        out.append(max(ek[max(0, n - W):n]) / peak if peak > 0.0 else 1.0)
    return np.array(out)


def _check_tracking():
    """Mismatches between the oracle's reported E_k, E_peak, residual and stop steps and their
    recomputation from its velocities."""
    bad = []
    body = _body()
    ob = oracle.OracleBody(body)
    W = ob.window
    assert W > 50 and SEG1 > 3 * W     # the window matters and the run outlasts it
    segments = []
    for seg_len in (SEG1, SEG2):
        ek_ref, ek_o, peak_o, res_o = [], [], [], []
        for _ in range(seg_len):
            ob.step(1)
            _, v = ob.get_state()
            ek_ref.append(_ek(body, v))
            ek_o.append(ob.kinetic_energy)
            peak_o.append(ob.ek_peak)
            res_o.append(ob.residual)
        segments.append((np.array(ek_ref), np.array(ek_o), np.array(peak_o), np.array(res_o)))
        # the tracking restarts on set_state (same state, same step index and dt)
        u, v = ob.get_state()
        ob.set_state(u, v, step=ob.step_index, dt=ob.dt)
    for s, (ek_ref, ek_o, peak_o, res_o) in enumerate(segments):
        if np.abs(ek_o - ek_ref).max() > 1e-15 * ek_ref.max():
            bad.append(f"segment {s}: E_k differs from 1/2 sum m|v|^2")
        peak_ref = np.maximum.accumulate(ek_ref)
        if np.abs(peak_o - peak_ref).max() > 1e-15 * peak_ref.max():
            bad.append(f"segment {s}: E_peak is not the running maximum of E_k")
        r_ref = _residuals(ek_ref, W)
        if np.abs(res_o - r_ref).max() > 1e-13:
            k = int(np.abs(res_o - r_ref).argmax())
            bad.append(f"segment {s}: residual at step {k + 1} is {res_o[k]:.6g}, window definition gives {r_ref[k]:.6g}")
    # stop steps of relax on fresh bodies against the first n with r_n < tol and n >= W
    r_ref = _residuals(segments[0][0], W)
    steps = np.arange(1, len(r_ref) + 1)
    for tol in STOP_TOLS:
        hit = np.flatnonzero((r_ref < tol) & (steps >= W))
        assert len(hit), f"the trace never reaches tol {tol}"
        expect = int(steps[hit[0]])
        ob2 = oracle.OracleBody(body)
        rep = ob2.relax(tol, SEG1)
        ob2.close()
        if not rep["converged"] or rep["steps"] != expect:
            bad.append(f"tol {tol}: relax stopped after {rep['steps']} steps (converged {rep['converged']}), "
                       f"the stop rule gives step {expect}")
    ob.close()
    return bad


def test_oracle_residual_tracking_matches_its_definition():
    assert _check_tracking() == []


def test_stop_with_tol_above_one_is_the_window_length():
    """r_n <= 1 always, so with tol > 1 only n >= W can stop the run: exactly at step W."""
    body = _body()
    ob = oracle.OracleBody(body)
    rep = ob.relax(1.5, 10 * ob.window)
    assert rep["converged"] and rep["steps"] == ob.window


# ---- planted mistakes (compiled into a private copy of the oracle, on the CPU) ----

MUTATIONS = {
    "current E_k instead of the window maximum": (
        "for (int64_t q = 0; q < b->win_fill; ++q) wmax = fmax(wmax, b->ek_win[q]);",
        "wmax = ek;"),
    "n >= W dropped from the stop rule": (
        "if (b->resid_last < tol && b->step >= b->win)",
        "if (b->resid_last < tol)"),
    "E_peak not raised when E_k grows": (
        "if (ek > b->ek_peak) b->ek_peak = ek;",
        "if (b->ek_peak == 0.0) b->ek_peak = ek;"),
}


@pytest.mark.parametrize("what", sorted(MUTATIONS))
def test_planted_mistake_is_caught(what, tmp_path, monkeypatch):
    old, new = MUTATIONS[what]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"the oracle no longer holds the line this mutation edits: {old}"
    path = tmp_path / "mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libmutant.so")
    subprocess.check_call(["gcc", *oracle.CFLAGS, "-o", so, str(path), "-lm"])
    monkeypatch.setattr(oracle, "_lib", oracle.load_library(so))
    assert _check_tracking() != [], what
    assert os.path.exists(so)


def test_divergence_rule_trips_where_its_definition_says():
    """Blow-up detection (a reading of the build; the paper has none): once E_k first falls below
    E_peak, a step whose E_k exceeds `factor` times that E_peak fails with E_DIVERGED.  The trip
    step is recomputed from the E_k series of the same run without the limit; the default factor
    (1e6) never trips on a relaxing body."""
    body = _body()
    ref = oracle.OracleBody(body)
    ek = []
    for _ in range(300):
        ref.step(1)
        ek.append(ref.kinetic_energy)
    ek = np.array(ek)
    peak = np.maximum.accumulate(ek)
    t = int(np.flatnonzero(ek < peak)[0])
    q = peak[t]
    factor = 2.0
    later = np.flatnonzero(ek[t:] > factor * q)
    assert len(later) and later[0] > 0, "the trace must cross factor x q after the turn-over step"
    expect = t + int(later[0]) + 1
    ob = oracle.OracleBody(body)
    ob.set_divergence(factor)
    with pytest.raises(oracle.OracleError) as e:
        ob.step(300)
    assert e.value.code == oracle.E_DIVERGED and ob.step_index == expect
    u, v = ob.get_state()
    assert np.isfinite(u).all() and np.isfinite(v).all()
    # the default factor: the same 300 steps run through
    ob2 = oracle.OracleBody(body)
    ob2.step(300)
    assert ob2.step_index == 300
