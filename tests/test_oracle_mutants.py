"""The pins are strong enough to catch plausible mistakes in the oracle.

Each case plants one mistake (a dropped term, a wrong sign, index or
boundary, a transposed operand, a changed order or definition) into a copy of
the oracle's C source, builds it with gcc into a temporary directory, binds
it in place of the oracle's library and runs the oracle pins in-process (cheap
ones first) until one fails.  A mistake that no pin catches fails the test.
Every planted mistake keeps the code memory-safe.
"""
import importlib
import inspect
import os
import subprocess

import pytest

import oracle

SRC = os.path.join(os.path.dirname(oracle.__file__), "rdseg_oracle.c")

# (name, exact text in the source, replacement); each text occurs exactly once
MUTANTS = [
    # discrete operators (end of Sec. 2.1)
    ("grad_x_sign", "gx[i] = (x < W - 1) ? u[i + 1] - u[i] : 0.0;",
     "gx[i] = (x < W - 1) ? u[i] - u[i + 1] : 0.0;"),
    ("grad_y_index", "gy[i] = (y < H - 1) ? u[i + W] - u[i] : 0.0;",
     "gy[i] = (y < H - 1) ? u[i + W] - u[i + 1] : 0.0;"),
    ("div_x_boundary", "if (x > 0) dx -= px[i - 1];", "if (x > 1) dx -= px[i - 1];"),
    ("div_y_transposed", "if (y > 0) dy -= py[i - W];", "if (y > 0) dy -= px[i - W];"),
    # active set (Sec. 3)
    ("rd_not_strict", "return fabs((double)fv) < delta;", "return fabs((double)fv) <= delta;"),
    ("heaviside_at_zero", "return ((double)fv < 0.0) ? 1.0 : 0.0;",
     "return ((double)fv <= 0.0) ? 1.0 : 0.0;"),
    ("clamp_no_upper", "(s > 1.0 ? 1.0 : s)", "(s > 1.0 ? s : s)"),
    # dual step (Sec. 3, restricted Chambolle step)
    ("w_sign", "c->w[i] = c->A[i] ? c->d[i] - v[i] / theta : -c->h[i] / theta;",
     "c->w[i] = c->A[i] ? c->d[i] + v[i] / theta : -c->h[i] / theta;"),
    ("frozen_w_zero", "c->w[i] = c->A[i] ? c->d[i] - v[i] / theta : -c->h[i] / theta;",
     "c->w[i] = c->A[i] ? c->d[i] - v[i] / theta : 0.0;"),
    ("norm_x_only", "c->qx[i] = (px[i] + tau * c->gx[i]) / (1.0 + tau * n);",
     "c->qx[i] = (px[i] + tau * c->gx[i]) / (1.0 + tau * fabs(c->gx[i]));"),
    ("dual_tau_dropped", "c->qy[i] = (py[i] + tau * c->gy[i]) / (1.0 + tau * n);",
     "c->qy[i] = (py[i] + c->gy[i]) / (1.0 + tau * n);"),
    # u-step, v-step, start and order (Sec. 2.1 / Sec. 3)
    ("u_step_sign", "if (c->A[i]) u[i] = v[i] - theta * c->d[i];",
     "if (c->A[i]) u[i] = v[i] + theta * c->d[i];"),
    ("v_step_theta_dropped", "if (c->A[i]) v[i] = clamp01(u[i] - theta * lambda * c->fd[i]);",
     "if (c->A[i]) v[i] = clamp01(u[i] - lambda * c->fd[i]);"),
    ("v0_unclamped",
     "                v[i] = clamp01(u[i] - theta * lambda * c->fd[i]);\n                px[i]",
     "                v[i] = u[i];\n                px[i]"),
    ("order_swapped",
     "        for (int j = 0; j < inner; ++j) dual_step(&c, theta, tau, v, px, py);\n"
     "        uv_step(&c, lambda, theta, px, py, u, v);\n    }\n    ctx_free(&c);",
     "        uv_step(&c, lambda, theta, px, py, u, v);\n"
     "        for (int j = 0; j < inner; ++j) dual_step(&c, theta, tau, v, px, py);\n"
     "    }\n    ctx_free(&c);"),
    # reverse mode
    ("reverse_norm_term_dropped", "double gbx = tau * m * pbx[i] - tau * m * dot * hx;",
     "double gbx = tau * m * pbx[i];"),
    ("reverse_theta_dropped", "                pbx[i] += theta * tx[i];",
     "                pbx[i] += tx[i];"),
    ("reverse_w_sign", "if (c.A[i]) vb[i] += -wb[i] / theta;", "if (c.A[i]) vb[i] += wb[i] / theta;"),
    # band threshold q-hat (Sec. 3) and the count behind it
    ("count_floor", "unsigned __int128 k = (prod + ((one << s) - 1)) >> s;",
     "unsigned __int128 k = prod >> s;"),
    ("qhat_not_above", "*qhat = nextafter(a[k - 1], INFINITY);", "*qhat = a[k - 1];"),
    # stopping rule and measures (Sec. 4)
    ("stop_strict", "if (d <= tol) break;", "if (d < tol) break;"),
    ("stop_u_only", "if (dv > d) d = dv;", "if (dv > d) d = d;"),
    ("union_as_intersection", "b += (g || o);", "b += (g && o);"),
    ("e2_absolute", "s += d * d;", "s += fabs(d);"),
    # volumes (Sec. 5 extension)
    ("grad3_z_index", "gz[i] = z < D - 1 ? u[i + (size_t)H * W] - u[i] : 0.0;",
     "gz[i] = z < D - 1 ? u[i + W] - u[i] : 0.0;"),
    ("norm3_z_dropped", "double n = sqrt(gx[i] * gx[i] + gy[i] * gy[i] + gz[i] * gz[i]);",
     "double n = sqrt(gx[i] * gx[i] + gy[i] * gy[i]);"),
    # primal-dual solver (Sec. 5 extension)
    ("pd_no_extrapolation", "ub[i] = 2.0 * un - u[i];", "ub[i] = un;"),
    ("pd_fit_sign", "double un = clamp01(u[i] + tau * c.d[i] - tau * lambda * c.fd[i]);",
     "double un = clamp01(u[i] + tau * c.d[i] + tau * lambda * c.fd[i]);"),
    ("pd_projection", "double s = n > 1.0 ? n : 1.0;", "double s = n + 1.0;"),
]

PIN_MODULES = ["tests.test_oracle_pins", "tests.test_oracle_band_stop", "tests.test_oracle_3d",
               "tests.test_oracle_pd", "tests.test_oracle_adjoint"]
SLOW = ("dense_projected", "duality_gap", "pd_duality_gap")


def _expand(fn):
    """Argument sets of a test function from its parametrize marks."""
    combos = [{}]
    for m in getattr(fn, "pytestmark", []):
        if m.name != "parametrize":
            continue
        names = m.args[0]
        names = [n.strip() for n in names.split(",")] if isinstance(names, str) else list(names)
        expanded = []
        for c in combos:
            for val in m.args[1]:
                if hasattr(val, "values") and hasattr(val, "marks"):
                    val = val.values if len(names) > 1 else val.values[0]
                vals = tuple(val) if len(names) > 1 else (val,)
                d = dict(c)
                d.update(zip(names, vals))
                expanded.append(d)
        combos = expanded
    return combos


def _pins():
    fast, slow = [], []
    for modname in PIN_MODULES:
        mod = importlib.import_module(modname)
        for name, fn in inspect.getmembers(mod, inspect.isfunction):
            if not name.startswith("test_") or fn.__module__ != modname:
                continue
            params = set(inspect.signature(fn).parameters)
            for kw in _expand(fn):
                if set(kw) != params:
                    continue   # needs a fixture: not run here
                (slow if any(s in name for s in SLOW) else fast).append(
                    (f"{modname.split('.')[-1]}::{name}{sorted(kw.items())}", fn, kw))
    return fast + slow


PINS = _pins()


def test_pins_collected():
    assert len(PINS) > 100


def test_unmutated_source_passes_every_pin():
    for label, fn, kw in PINS:
        fn(**kw)


@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_planted_mistake(name, old, new, tmp_path):
    src = open(SRC).read()
    assert src.count(old) == 1, f"{name}: the text to replace must occur exactly once"
    mutant = tmp_path / f"mutant_{name}.c"
    mutant.write_text(src.replace(old, new))
    lib = tmp_path / f"libmutant_{name}.so"
    subprocess.run(["gcc", "-O1", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared", "-w",
                    "-o", str(lib), str(mutant), "-lm"], check=True)
    saved = oracle._lib
    oracle._lib = oracle._bind(str(lib))
    caught = None
    try:
        for label, fn, kw in PINS:
            try:
                fn(**kw)
            except Exception as e:   # an assertion, or an error the mistake provoked
                caught = (label, type(e).__name__)
                break
    finally:
        oracle._lib = saved
    assert caught is not None, f"no pin catches the planted mistake {name}"
