"""Helpers shared by the GPU parity tests: seeded inputs on the device, the same
inputs handed to the oracle on the host."""
import math
import sys

import numpy as np
import torch

import oracle as O
import synth


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device_linelist(cfg, n_lines=None, n_states=None, device="cuda"):
    d = synth.make_linelist(cfg, n_lines=n_lines, n_states=n_states, device=device)
    return d


def host(d):
    return {k: v.detach().cpu().numpy() for k, v in d.items()}


def make_plan(cfg, precision="fp32", profile="voigt", **kw):
    from paper_1801_09803_amd import Plan
    return Plan(cfg.nu_a, cfg.nu_b, cfg.n_points, cfg.mass_amu, cutoff=cfg.cutoff,
                profile=profile, precision=precision, **kw)


def oracle_lineset(h, cfg, T, P, **kw):
    return O.make_lineset(h["E"], h["g"], h["upper"], h["lower"], h["A"], T, P, cfg.mass_amu,
                          gamma_ref=h["gamma_ref"], n_exp=h["n_exp"], **kw)


def assert_parity(got, ref, tol, area_tol=None, what=""):
    m = O.error_metrics(got, ref)
    log(f"  parity {what}: max_rel={m['max_rel']:.3e} area_rel={m['area_rel']:.3e} n={m['n_checked']}")
    assert m["n_checked"] > 0
    assert m["max_rel"] <= tol, (what, m)
    assert m["area_rel"] <= (tol if area_tol is None else area_tol), (what, m)
    return m
