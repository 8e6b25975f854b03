"""Planted mistakes in the oracle (CPU only): each mutant of mgfr_oracle.c must fail at
least one pin in test_oracle_pins.py or test_masked_oracle.py, so a plausible slip anywhere in the oracle (a dropped
term, a wrong sign, a wrong weight or exponent) cannot pass unnoticed."""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "mgfr_oracle.c")

MUTANTS = {
    "density coefficient Om a / 3": (
        "L -= c->D * (g->rho[at(n, i, j, k)] - g->rho_ref) + c->Sbar;",
        "L -= c->D / 3.0 * (g->rho[at(n, i, j, k)] - g->rho_ref) + c->Sbar;"),
    "sign of b_nb in the Jacobian": (
        "dL += g->C * (bi * (un - ui) - bn - bi);",
        "dL += g->C * (bi * (un - ui) + bn - bi);"),
    "ghost b interpolated linearly": (
        "double bg = exp(ug);",
        "double bg = (1.0 - g->r) * exp(ubv) + g->r * bi;"),
    "prolongation face weight 3/64": (
        "9.0 / 64.0 * (coarse_val(nc, v, periodic, I + si, J, K) +",
        "3.0 / 64.0 * (coarse_val(nc, v, periodic, I + si, J, K) +"),
    "FAS right-hand side sign": (
        "H->f[q] = cell_op(&H->g, c, H->uhat, I, J, K, NULL) - H->f[q];",
        "H->f[q] = cell_op(&H->g, c, H->uhat, I, J, K, NULL) + H->f[q];"),
    "curvature exponent 1/(n+2)": (
        "double S = c->A * exp(-ui / (c->n + 1.0));",
        "double S = c->A * exp(-ui / (c->n + 2.0));"),
    "background exponent n": (
        "c->ubar = log(n * a * a * c->xi / pow(3.0 * q, n + 1.0));",
        "c->ubar = log(n * a * a * c->xi / pow(3.0 * q, n));"),
    "xi without 1/n": (
        "c->xi = m->fr0_abs * pow(3.0 * (1.0 + 4.0 * ol / om), n + 1.0) / n;",
        "c->xi = m->fr0_abs * pow(3.0 * (1.0 + 4.0 * ol / om), n + 1.0);"),
    "face b without b_i": (
        "L += g->C * (bn + bi) * (un - ui);",
        "L += g->C * (bn + bn) * (un - ui);"),
    "boundary value = ghost value": (
        "ub[((long long)f * n + p) * n + q] = (ug - r * ui) / (1.0 - r);",
        "ub[((long long)f * n + p) * n + q] = ug;"),
    "restriction weight 1/7": (
        "coarse[at(nc, I, J, K)] = s / 8.0;",
        "coarse[at(nc, I, J, K)] = s / 7.0;"),
    "ghost Jacobian without r": (
        "dL += g->C * ((g->r * bg + bi) * (ug - ui) + (bg + bi) * (g->r - 1.0));",
        "dL += g->C * ((bg + bi) * (ug - ui) + (bg + bi) * (g->r - 1.0));"),
    # the refinement level with the mask scheme
    "masked boundary value = fixed neighbour value": (
        "double ubv = (mi * g->w[p] - mn * g->w[q]) / (mi - mn);",
        "double ubv = g->w[p];"),
    "masked ghost without r u_i": (
        "double r = mn / mi;",
        "double r = 0.0 * mn / mi;"),
    "masked ghost Jacobian without r": (
        "dL += g->C * ((r * bg + bi) * (ug - ui) + (bg + bi) * (r - 1.0));",
        "dL += g->C * ((bg + bi) * (ug - ui) + (bg + bi) * (r - 1.0));"),
    "masked cells relaxed too": (
        "if (!(g->mask[q] > 0.0)) continue;\n                    double d;",
        "if (!(g->mask[q] > -2.0)) continue;\n                    double d;"),
    "correction prolongated into masked cells": (
        "if (F->g.mask[q] > 0.0) F->u[q] += corr[q];",
        "F->u[q] += corr[q];"),
    "masked FAS right-hand side sign": (
        "masked_op(&H->g, c, H->uhat, I, J, K, NULL) - Rd[q]",
        "masked_op(&H->g, c, H->uhat, I, J, K, NULL) + Rd[q]"),
    "masked prolongation without the coarse correction": (
        "H->d[q] = H->g.mask[q] > 0.0 ? H->u[q] - H->uhat[q] : 0.0;",
        "H->d[q] = 0.0;"),
}

PIN_FILES = ("test_oracle_pins.py", "test_masked_oracle.py")


def _run(name, old, new, tmpdir):
    src = open(SRC).read()
    assert old in src, name
    tag = "".join(ch if ch.isalnum() else "_" for ch in name)
    c = os.path.join(tmpdir, tag + ".c")
    so = os.path.join(tmpdir, tag + ".so")
    with open(c, "w") as f:
        f.write(src.replace(old, new, 1))
    subprocess.check_call(["gcc", "-O2", "-shared", "-fPIC", "-I", os.path.join(ROOT, "oracle"), c, "-o", so, "-lm"])
    env = dict(os.environ, MGFR_ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] +
                       [os.path.join(ROOT, "tests", f) for f in PIN_FILES],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_fails_a_pin(tmp_path):
    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(lambda kv: _run(kv[0], kv[1][0], kv[1][1], str(tmp_path)), MUTANTS.items()))
    survivors = [n for n, rc in results if rc == 0]
    assert not survivors, f"mutants not caught by any pin: {survivors}"
