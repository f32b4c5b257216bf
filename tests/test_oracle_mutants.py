"""Planted mistakes in a copy of the oracle must fail its pins.

The pins in the other ``test_oracle_*`` files check the oracle against what
the mathematics fixes (closed forms, exact solutions, identities, symmetries,
convergence orders).  This file checks that they are strong enough: each case
copies ``oracle/`` and ``tests/`` into a temporary root, changes one
expression of the copy's arithmetic (a sign, an index, a dropped term or
factor, a transposed operand, a wrong constant), rebuilds the copy and runs
the pin files that cover that code in a child process, which imports the
copy.  A case passes when that child run fails.  An unchanged copy must pass
the same files, so that a failure comes from the planted mistake and not
from the harness.  Nothing here touches the oracle in the repository, and
every planted change keeps all array accesses in bounds.
"""
import concurrent.futures
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

RP = ["test_oracle_rp.py", "test_oracle_step.py"]
STEP = ["test_oracle_step.py"]
STRANG = ["test_oracle_strang.py"]
UNSPLIT = ["test_oracle_unsplit.py"]
AMR = ["test_oracle_amr.py"]
SUR = ["test_oracle_surrogate.py"]

# (name, file under oracle/, text, replacement, pin files)
MUTANTS = [
    # Riemann solvers
    ("sw_alpha3_sign", "mco.c",
     "double a3 = (d1 - (uhat - chat) * d0) / (2.0 * chat);",
     "double a3 = (d1 + (uhat - chat) * d0) / (2.0 * chat);", RP),
    ("sw_roe_average_unweighted", "mco.c",
     "double uhat = (sql * ul + sqr * ur) / (sql + sqr);",
     "double uhat = 0.5 * (ul + ur);", RP),
    ("sw_entropy_fix_dropped", "mco.c",
     "double f = lam_l * (lam_r - s[0]) / (lam_r - lam_l);",
     "double f = s[0] < 0.0 ? s[0] : 0.0;", RP),
    ("sw_shear_wave_transposed", "mco.c",
     "W2[0] = 0.0; W2[mu] = 0.0; W2[mv] = a2;",
     "W2[0] = 0.0; W2[mu] = a2; W2[mv] = 0.0;", RP),
    ("acoustics_impedance_inverted", "mco.c",
     "double Z = P->rho * c;",
     "double Z = P->rho / c;", RP),
    ("vc_acoustics_impedances_swapped", "mco.c",
     "double a1 = (-dp + zr * du) / (zl + zr);",
     "double a1 = (-dp + zl * du) / (zl + zr);", RP),
    ("sw_depth_average_geometric", "mco.c",
     "double hbar = 0.5 * (hl + hr);",
     "double hbar = sqrt(hl * hr);", RP),
    ("euler_hlle_left_bound_reversed", "mco.c",
     "sL = ul - cl; if (uhat - chat < sL) sL = uhat - chat;",
     "sL = ul - cl; if (uhat - chat > sL) sL = uhat - chat;", RP),
    ("euler_pressure_gamma", "mco.c",
     "return (gm - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);",
     "return gm * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);", RP),
    ("euler_entropy_strength_sign", "mco.c",
     "+ vhat * d2 - d3);",
     "+ vhat * d2 + d3);", RP),
    ("euler_eigenvector_energy_sign", "mco.c",
     "W4[3] = a4 * (Hhat + uhat * chat);",
     "W4[3] = a4 * (Hhat - uhat * chat);", RP),
    # limiter, correction flux, update, CFL
    ("mc_limiter_half_dropped", "mco.c",
     "double c = 0.5 * (1.0 + theta);",
     "double c = (1.0 + theta);", STEP),
    ("minmod_clamp_at_two", "mco.c",
     "r = theta < 1.0 ? theta : 1.0;",
     "r = theta < 2.0 ? theta : 2.0;", STEP),
    ("superbee_second_branch_clamp", "mco.c",
     "double b = theta < 2.0 ? theta : 2.0;",
     "double b = theta < 1.0 ? theta : 1.0;", STEP),
    ("van_leer_denominator", "mco.c",
     "return (theta + fabs(theta)) / (1.0 + fabs(theta));",
     "return (theta + fabs(theta)) / (2.0 + fabs(theta));", STEP),
    ("limiter_downwind_neighbour", "mco.c",
     "int kk = (sp > 0.0) ? k - 1 : k + 1;",
     "int kk = (sp > 0.0) ? k + 1 : k - 1;", STEP),
    ("correction_factor_sign", "mco.c",
     "double c = 0.5 * fabs(sp) * (1.0 - nu * fabs(sp));",
     "double c = 0.5 * fabs(sp) * (1.0 + nu * fabs(sp));", STEP),
    ("update_correction_sign", "mco.c",
     "- nu * (W->ftil[m * ne + kr] - W->ftil[m * ne + kl]);",
     "+ nu * (W->ftil[m * ne + kr] - W->ftil[m * ne + kl]);", STEP),
    ("update_fluctuations_swapped", "mco.c",
     "double v = qi - nu * (W->apdq[m * ne + kl] + W->amdq[m * ne + kr])",
     "double v = qi - nu * (W->amdq[m * ne + kl] + W->apdq[m * ne + kr])", STEP),
    ("cfl_division_dropped", "mco.c",
     "double v = fabs(W->s[p * ne + k]) / d;",
     "double v = fabs(W->s[p * ne + k]);", STEP),
    # boundary rule, the split step, the time-step rule
    ("extrapolation_right_ghost_index", "mco.c",
     "return i < 0 ? 0 : (i >= n ? n - 1 : i);",
     "return i < 0 ? 0 : (i >= n ? 0 : i);", STEP),
    ("y_sweep_courant_from_dx", "mco.c",
     "st |= sweep2d(solver, P, 2, nx, ny, g, ga, dt / dy, dy, limiter, qout, &sy, nthreads);",
     "st |= sweep2d(solver, P, 2, nx, ny, g, ga, dt / dx, dy, limiter, qout, &sy, nthreads);", STEP),
    ("boundary_rule_not_reapplied", "mco.c",
     "fill_ghosts(meqn, nx, ny, qs, bc, g);",
     "fill_ghosts(meqn, nx, ny, qs, MCO_BC_PERIODIC, g);", STEP),
    ("dt_rule_halves_after_rejection", "mco.c",
     "dt = cfl_target / sm;",
     "dt = 0.5 * dt;", STEP),
    ("dt_rule_never_rejects", "mco.c",
     "if (cfl > cfl_max) {",
     "if (cfl > 1e300) {", STEP),
    ("fluctuation_split_at_zero", "mco.c",
     "double sp = s[p] > 0.0 ? s[p] : 0.0;",
     "double sp = s[p] >= 0.0 ? s[p] : s[p];", RP),
    ("hlle_middle_state_flux_sign", "mco.c",
     "qs[m] = (sR * qr[m] - sL * ql[m] - (fr[m] - fl[m])) / (sR - sL);",
     "qs[m] = (sR * qr[m] - sL * ql[m] + (fr[m] - fl[m])) / (sR - sL);", RP),
    ("sw_flux_hydrostatic_half_dropped", "mco.c",
     "f[mu] = q[mu] * un + 0.5 * g * h * h;",
     "f[mu] = q[mu] * un + g * h * h;", RP),
    ("sw_hlle_right_bound_reversed", "mco.c",
     "if (uhat + chat > sR) sR = uhat + chat;",
     "if (uhat + chat < sR) sR = uhat + chat;", RP),
    ("euler_flux_energy_pressure_dropped", "mco.c",
     "f[3] = (q[3] + p) * un;",
     "f[3] = q[3] * un;", RP),
    ("euler_entropy_fix_family4_speed", "mco.c",
     "double lam_l = q3[mu] / q3[0] + sqrt(gm * p3 / q3[0]);",
     "double lam_l = q3[mu] / q3[0] - sqrt(gm * p3 / q3[0]);", RP),
    # the oracle's array marshalling
    ("binding_dx_dy_swapped", "__init__.py",
     "st = lib().mco_step2d(solver, ctypes.byref(P), nx, ny, dx, dy, _p(q), _p(auxa), dt,",
     "st = lib().mco_step2d(solver, ctypes.byref(P), nx, ny, dy, dx, _p(q), _p(auxa), dt,", STEP),
    ("binding_grid_transposed", "__init__.py",
     "    meqn, ny, nx = q.shape\n    auxa = _f64(aux) if aux is not None else None\n    out = np.empty_like(q)\n    sm = ctypes.c_double(0.0)\n    st = lib().mco_step2d(",
     "    meqn, nx, ny = q.shape\n    auxa = _f64(aux) if aux is not None else None\n    out = np.empty_like(q)\n    sm = ctypes.c_double(0.0)\n    st = lib().mco_step2d(", STEP),
    # Strang splitting
    ("strang_full_first_half_step", "strang.py",
     "q1, s1 = sweep(solver, P, q, aux, 1, 0.5 * dt / dx, limiter, bc)",
     "q1, s1 = sweep(solver, P, q, aux, 1, dt / dx, limiter, bc)", STRANG),
    ("strang_smax_half_dropped", "strang.py",
     "return q3, max(0.5 * s1 / dx, s2 / dy, 0.5 * s3 / dx)",
     "return q3, max(s1 / dx, s2 / dy, s3 / dx)", STRANG),
    # unsplit step with transverse solves
    ("unsplit_transverse_factor", "unsplit.py",
     "half = 0.5 * nux",
     "half = nux", UNSPLIT),
    ("unsplit_sw_transverse_strength_sign", "unsplit.py",
     "b3 = (d[t] - (ut - c) * d[0]) / (2.0 * c)",
     "b3 = (d[t] + (ut - c) * d[0]) / (2.0 * c)", UNSPLIT),
    ("unsplit_transverse_wrong_edge", "unsplit.py",
     "F[:, 1:, :] -= halfy * ybpAp[:, :, :-1]",
     "F[:, :-1, :] -= halfy * ybpAp[:, :, :-1]", UNSPLIT),
    ("unsplit_acoustics_transverse_speed_sign", "unsplit.py",
     "return -c * b1 * r1, c * b3 * r3",
     "return c * b1 * r1, c * b3 * r3", UNSPLIT),
    ("unsplit_vc_transverse_impedance", "unsplit.py",
     "g2 = (d[0] + Zm * d[t]) / (Zm + Za)",
     "g2 = (d[0] + Za * d[t]) / (Zm + Za)", UNSPLIT),
    ("unsplit_euler_transverse_strength", "unsplit.py",
     "b3 = d[n] - un * d[0]",
     "b3 = d[n] - ut * d[0]", UNSPLIT),
    # two-level refinement coupling
    ("amr_reflux_sign", "amr.py",
     "q = q + nux * (Fbar - Fc)",
     "q = q - nux * (Fbar - Fc)", AMR),
    ("amr_no_time_interpolation", "amr.py",
     "vals[:, unc] = (1.0 - alpha) * a + alpha * b",
     "vals[:, unc] = a", AMR),
    ("amr_interpolation_offset", "amr.py",
     "xi = ((I % r) + 0.5) / r - 0.5",
     "xi = (I % r) / r - 0.5", AMR),
    ("amr_fine_flux_average", "amr.py",
     "Fbar = s / (r * r)",
     "Fbar = s / r", AMR),
    # learned edge solver
    ("gelu_cubic_coefficient", "surrogate.py",
     "GELU_A = 0.044715",
     "GELU_A = 0.0447", SUR),
    ("adam_bias_correction_dropped", "surrogate.py",
     "mh = m / (1.0 - b1 ** t)",
     "mh = m", SUR),
    ("features_velocity_not_scaled", "surrogate.py",
     "X = np.stack([ub / c0, vb / c0, m, e[0], e[1], e[2]], axis=1)",
     "X = np.stack([ub, vb / c0, m, e[0], e[1], e[2]], axis=1)", SUR),
    ("adam_second_moment_coefficient", "surrogate.py",
     "v = b2 * v + (1.0 - b2) * grad * grad",
     "v = b2 * v + (1.0 - b1) * grad * grad", SUR),
    ("fallback_flag_family3_sign", "surrogate.py",
     "l3l = q2[1] / h2 + np.sqrt(g * h2)",
     "l3l = q2[1] / h2 - np.sqrt(g * h2)", SUR),
    ("projection_speed_factor_dropped", "surrogate.py",
     "Wp = np.stack([W[p] + s[p] * r / Dn for p in range(s.shape[0])])",
     "Wp = np.stack([W[p] + r / Dn for p in range(s.shape[0])])", SUR),
]

CONTROL = ("unchanged", None, None, None, sorted(set(RP + STEP + STRANG + UNSPLIT + AMR + SUR)))


def _ignore(_dir, names):
    return [n for n in names if n == "__pycache__" or n.endswith(".tmp")]


def _run(base, case):
    name, fname, old, new, pins = case
    root = os.path.join(base, name)
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(root, "oracle"), ignore=_ignore)
    shutil.copytree(os.path.join(ROOT, "tests"), os.path.join(root, "tests"), ignore=_ignore)
    if fname is not None:
        path = os.path.join(root, "oracle", fname)
        src = open(path).read()
        if src.count(old) < 1:
            return name, "harness", f"text to change not found in oracle/{fname}: {old!r}"
        with open(path, "w") as f:
            f.write(src.replace(old, new, 1))
        if fname.endswith(".c"):
            lib = os.path.join(root, "oracle", "liboracle.so")
            if os.path.exists(lib):
                os.remove(lib)
            b = subprocess.run([sys.executable, os.path.join(root, "oracle", "build.py")],
                               capture_output=True, text=True, timeout=300)
            if b.returncode != 0:
                return name, "harness", "build failed:\n" + b.stderr[-2000:]
    env = dict(os.environ)
    # the copy's tests put the copy's root first on sys.path (their conftest);
    # the input generators come from the repository
    env["PYTHONPATH"] = ROOT + os.pathsep + env.get("PYTHONPATH", "")
    env["OMP_NUM_THREADS"] = "1"
    cmd = [sys.executable, "-m", "pytest", "-x", "-q", "-m", "not gpu", "-p", "no:cacheprovider"] + \
        [os.path.join(root, "tests", p) for p in pins]
    r = subprocess.run(cmd, capture_output=True, text=True, cwd=root, env=env, timeout=600)
    tail = (r.stdout + r.stderr)[-3000:]
    if r.returncode == 0:
        return name, "passed", tail
    if r.returncode == 1:
        return name, "failed", tail
    return name, "harness", f"child pytest exit code {r.returncode}:\n{tail}"


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    import oracle
    if not os.path.exists(oracle.LIBPATH):
        from oracle import build
        build.build()
    base = str(tmp_path_factory.mktemp("mutants"))
    cases = [CONTROL] + MUTANTS
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        out = list(ex.map(lambda c: _run(base, c), cases))
    return {name: (verdict, tail) for name, verdict, tail in out}


def test_unchanged_copy_passes_its_pins(results):
    verdict, tail = results["unchanged"]
    assert verdict == "passed", tail


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_planted_mistake_fails_a_pin(results, name):
    verdict, tail = results[name]
    assert verdict != "harness", tail
    assert verdict == "failed", f"planted mistake {name} passed every pin:\n{tail}"
