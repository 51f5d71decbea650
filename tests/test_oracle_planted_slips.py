"""Planted slips: every pin must catch a plausible mistake in the oracle.

Each entry below plants one mistake (a text substitution) in a scratch copy of
``oracle/lbpo.c``, builds it with the oracle's own compiler flags, and runs the
named pins against that build in a child process (``LBPO_LIB`` points the
oracle's loader at it).  The pins must fail; the unmodified copy must pass
them.  Nothing here touches the committed oracle or the GPU library.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
BP = "tests/test_oracle_boundary_pins.py"
PINS = "tests/test_oracle_pins.py"

# (name, original text, planted text, pin file, -k expression of the pins
# that must fail).  The original text must occur exactly once.
SLIPS = [
    # open sides (Sec. IV.A outer boundary; reading of the open rule)
    ("open f: bounce-back instead of the zero-gradient copy",
     "      fn = h->fp[a * n + gh.idx];\n      gn = h->wg[a] * gh.T;",
     "      fn = h->fp[OPP[a] * n + i];\n      gn = h->wg[a] * gh.T;",
     BP, "pass_a_uniform_flow"),
    ("open g: anti-bounce-back instead of the rest equilibrium",
     "      gn = h->wg[a] * gh.T;",
     "      gn = -h->gp[OPP[a] * n + i] + 2.0 * h->wg[a] * gh.T;",
     BP, "conduction_profile"),
    ("open g: copied from the clamped source",
     "      gn = h->wg[a] * gh.T;", "      gn = h->gp[a * n + gh.idx];",
     BP, "conduction_profile"),
    ("open g: D2Q9 weights instead of the Eq. (53) rest weights",
     "      gn = h->wg[a] * gh.T;", "      gn = WL[a] * gh.T;",
     BP, "conduction_profile"),
    ("open stencil ghost: v = 0 as at a wall",
     "  return gh.kind == G_WALL ? 0.0 : h->ux[gh.idx];",
     "  return gh.kind != G_INSIDE ? 0.0 : h->ux[gh.idx];",
     BP, "ghosts_in_the_thermal_source"),
    ("open stencil ghost: T of the nearest node",
     "  return gh.kind == G_INSIDE ? h->T[gh.idx] : gh.T;",
     "  return gh.kind != G_WALL ? h->T[gh.idx] : gh.T;",
     BP, "ghosts_in_the_thermal_source"),
    ("open stencil ghost: rho = 0",
     "static double nb_rho(const lbpo_handle *h, ghost_t gh) { return "
     "h->rho[gh.idx]; }",
     "static double nb_rho(const lbpo_handle *h, ghost_t gh) { return "
     "gh.kind == G_OPEN ? 0.0 : h->rho[gh.idx]; }",
     BP, "ghosts_in_the_thermal_source"),
    ("open stencil ghost: psi = 0",
     "  if (gh.kind != G_WALL || (c->wet_amp == 0.0",
     "  if (gh.kind == G_OPEN) return 0.0;\n"
     "  if (gh.kind != G_WALL || (c->wet_amp == 0.0",
     BP, "pass_a_uniform_flow"),
    # hot spot (Sec. IV.B)
    ("hot spot: columns off by one",
     "col >= h->c.hot_x0 && col < h->c.hot_x1",
     "col > h->c.hot_x0 && col <= h->c.hot_x1",
     BP, "hot_spot_first_step_temperature"),
    ("hot spot: diagonal links take the destination column",
     "    ghost_t gh = resolve(h, x - EX[a], y - EY[a]);",
     "    ghost_t gh = resolve(h, x - EX[a], y - EY[a]);\n"
     "    if (gh.kind == G_WALL && y - EY[a] < 0) gh.T = side_T(h, 2, x);",
     BP, "hot_spot_first_step_temperature"),
    ("hot spot: diagonal links take the mirrored column",
     "    ghost_t gh = resolve(h, x - EX[a], y - EY[a]);",
     "    ghost_t gh = resolve(h, x - EX[a], y - EY[a]);\n"
     "    if (gh.kind == G_WALL && y - EY[a] < 0)\n"
     "      gh.T = side_T(h, 2, (x + EX[a] + h->nx) % h->nx);",
     BP, "hot_spot_first_step_temperature"),
    ("hot spot: stencil ghosts take the node's column",
     "    double Tn = nb_T(h, gh);",
     "    double Tn = nb_T(h, gh);\n"
     "    if (gh.kind == G_WALL && y + EY[a] < 0) Tn = side_T(h, 2, x);",
     BP, "hot_spot_first_step_source"),
    ("hot spot: on the y+ wall", "  if (side == 2 && col",
     "  if (side == 3 && col", BP, "hot_spot_first_step_temperature"),
    # corners: the wall wins, the y side gives the temperature
    ("corner: an open side wins over a wall",
     "    if ((ys >= 0 && h->c.bc[ys] == LBPO_BC_WALL) ||\n"
     "        (xs >= 0 && h->c.bc[xs] == LBPO_BC_WALL))",
     "    if ((ys >= 0 && h->c.bc[ys] == LBPO_BC_WALL) &&\n"
     "        (xs < 0 || h->c.bc[xs] == LBPO_BC_WALL))",
     BP, "corner_first_step_temperature"),
    ("corner: the x side gives the temperature",
     "    gh.T = ys >= 0 ? side_T(h, ys, x) : side_T(h, xs, x);",
     "    gh.T = xs >= 0 ? side_T(h, xs, x) : side_T(h, ys, x);",
     BP, "corner_first_step"),
    # buoyancy (Sec. IV.B)
    ("buoyancy: sign flipped",
     "      Fy += (h->rho[i] - h->rho_ave) * c->gy;",
     "      Fy -= (h->rho[i] - h->rho_ave) * c->gy;",
     BP, "buoyancy"),
    ("buoyancy: rho g without rho_ave",
     "      Fy += (h->rho[i] - h->rho_ave) * c->gy;",
     "      Fy += h->rho[i] * c->gy;",
     BP, "buoyancy_first_step_momentum"),
    ("buoyancy: rho_ave - rho",
     "      Fy += (h->rho[i] - h->rho_ave) * c->gy;",
     "      Fy += (h->rho_ave - h->rho[i]) * c->gy;",
     BP, "buoyancy"),
    # diagnostics (radius and energy readings)
    ("radius: pi outside the square root",
     "  d->radius = sqrt(d->liquid_area / M_PI);",
     "  d->radius = sqrt(d->liquid_area) / M_PI;",
     BP, "radius_of_a_tanh_disk"),
    ("radius: square root dropped",
     "  d->radius = sqrt(d->liquid_area / M_PI);",
     "  d->radius = d->liquid_area / M_PI;",
     BP, "radius_of_a_tanh_disk"),
    ("liquid area: upper clamp dropped",
     "    if (frac > 1.0) frac = 1.0;\n", "",
     BP, "clamps_and_threshold"),
    ("liquid area: lower clamp dropped",
     "    if (frac < 0.0) frac = 0.0;\n", "",
     BP, "clamps_and_threshold"),
    ("count radius: threshold at rho_l",
     "    if (r > half) count += 1.0;", "    if (r > h->c.rho_l) count += 1.0;",
     BP, "clamps_and_threshold"),
    ("liquid fraction: relative to rho_l",
     "    double frac = (r - h->c.rho_v) / (h->c.rho_l - h->c.rho_v);",
     "    double frac = r / h->c.rho_l;",
     BP, "radius_of_a_tanh_disk or clamps_and_threshold"),
    ("sum rho c_V T: c_V dropped",
     "    d->sum_rhocvT += r * h->c.cv * h->T[i];",
     "    d->sum_rhocvT += r * h->T[i];",
     BP, "sums_and_max_speed"),
    ("max |v|: one component only",
     "    double sp = sqrt(h->ux[i] * h->ux[i] + h->uy[i] * h->uy[i]);",
     "    double sp = fabs(h->ux[i]);",
     BP, "max_speed"),
    # earlier pins (Eqs. 28, 46, 53-56, the flow model, walls)
    ("Eq. (46): sign of the d_t phi term",
     "      h->S0[i] = h->phi[i] + 0.5 * (h->phi[i] - prev);",
     "      h->S0[i] = h->phi[i] - 0.5 * (h->phi[i] - prev);",
     PINS, "temperature_budget"),
    ("Eq. (46): 1 instead of 1/2",
     "      h->S0[i] = h->phi[i] + 0.5 * (h->phi[i] - prev);",
     "      h->S0[i] = h->phi[i] + 1.0 * (h->phi[i] - prev);",
     PINS, "temperature_budget"),
    ("Eq. (54): s3 in place of s4",
     "ms[3] += (1.0 - 0.5 * c->s_g[3]) * c->s_g[4] * (m[4] - meq[4]);",
     "ms[3] += (1.0 - 0.5 * c->s_g[3]) * c->s_g[3] * (m[4] - meq[4]);",
     PINS, "anisotropic_error and 0-1.4"),
    ("Eq. (54): (1 - s3/2) dropped",
     "ms[3] += (1.0 - 0.5 * c->s_g[3]) * c->s_g[4] * (m[4] - meq[4]);",
     "ms[3] += c->s_g[4] * (m[4] - meq[4]);",
     PINS, "anisotropic_error and 0-1.0"),
    ("Eq. (55) dropped",
     "        ms[5] += (1.0 - 0.5 * c->s_g[5]) * c->s_g[6] * (m[6] - meq[6]);",
     "", PINS, "anisotropic_error and 1-1.0"),
    ("Eq. (53): m2^eq = T", "  out[2] = 2.0 * T;", "  out[2] = T;",
     PINS, "eq44 or eq53"),
    ("Eq. (28): sign of the (dp/dT) term",
     "  return div_lam_gradT / rcv - h->k_th * lapT +\n"
     "         T * (1.0 - lbpo_dpdT(c, rho, T) / rcv) * divv;",
     "  return div_lam_gradT / rcv - h->k_th * lapT +\n"
     "         T * (1.0 + lbpo_dpdT(c, rho, T) / rcv) * divv;",
     PINS, "compressive_flow"),
    ("Eq. (28): grad lambda . grad T dropped",
     "  double div_lam_gradT = lam * lapT + (dlam_x * dTx + dlam_y * dTy);",
     "  double div_lam_gradT = lam * lapT;",
     PINS, "variable_conductivity"),
    ("Eq. (28): +k instead of -k",
     "  return div_lam_gradT / rcv - h->k_th * lapT +",
     "  return div_lam_gradT / rcv + h->k_th * lapT +",
     PINS, "gaussian_diffusion"),
    ("Eq. (56): sign of d theta / dT",
     "  return 2.0 * s * (-kappa) * (0.5 / sqrt(T * Tc));",
     "  return 2.0 * s * kappa * (0.5 / sqrt(T * Tc));",
     PINS, "dpdT_is_derivative"),
    ("velocity: F instead of F/2",
     "      h->ux[i] = (h->jx[i] + 0.5 * Fx) / h->rho[i];",
     "      h->ux[i] = (h->jx[i] + Fx) / h->rho[i];",
     BP, "momentum_gain"),
    ("forcing: half the force on jx", "        S[3] = Fx;",
     "        S[3] = 0.5 * Fx;", BP, "momentum_gain"),
    ("M: a swapped entry in the qx row",
     "    {0, -2, 0, 2, 0, 1, -1, -1, 1},      /* qx  */",
     "    {0, -2, 0, 2, 0, 1, -1, 1, -1},      /* qx  */",
     PINS, "M_rows_orthogonal"),
    ("wall g: bounce-back instead of anti-bounce-back",
     "      gn = -h->gp[OPP[a] * n + i] + 2.0 * h->wg[a] * gh.T;",
     "      gn = h->gp[OPP[a] * n + i];",
     PINS, "dirichlet_walls"),
    ("sigma term: + 1/2 in its denominator",
     "12.0 * c->sigma * Fm2 / (psi2 * (1.0 / c->s_f[1] - 0.5));",
     "12.0 * c->sigma * Fm2 / (psi2 * (1.0 / c->s_f[1] + 0.5));",
     PINS, "flat_interface"),
    ("interaction force: sign",
     "      double Fx = -c->G * h->psi[i] * sx;\n"
     "      double Fy = -c->G * h->psi[i] * sy;",
     "      double Fx = c->G * h->psi[i] * sx;\n"
     "      double Fy = c->G * h->psi[i] * sy;",
     PINS, "flat_interface"),
]


def _build(tmp, name, src):
    d = os.path.join(tmp, name)
    os.makedirs(d)
    shutil.copy(os.path.join(ORACLE, "lbpo.h"), d)
    with open(os.path.join(d, "lbpo.c"), "w") as f:
        f.write(src)
    lib = os.path.join(d, "liblbpo.so")
    subprocess.check_call(
        ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
         "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-o", lib,
         os.path.join(d, "lbpo.c"), "-lm"], cwd=d)
    return lib


def _run_pins(lib, pin_file, expr):
    env = dict(os.environ, LBPO_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run(
        [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
         "-p", "no:xdist", pin_file, "-k", expr], cwd=ROOT, env=env,
        capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_planted_slips_are_caught(tmp_path):
    with open(os.path.join(ORACLE, "lbpo.c")) as f:
        clean = f.read()
    jobs = []
    for k, (name, old, new, pin_file, expr) in enumerate(SLIPS):
        assert clean.count(old) == 1, f"slip text not unique: {name}"
        jobs.append((f"slip{k:02d}", clean.replace(old, new), pin_file, expr,
                     name))
    # the unmodified copy passes every selected pin
    base = _build(str(tmp_path), "clean", clean)
    for pin_file in (BP, PINS):
        exprs = sorted({e for _, _, p, e, _ in jobs if p == pin_file})
        rc, out = _run_pins(base, pin_file, " or ".join(f"({e})" for e in exprs))
        assert rc == 0, f"clean oracle fails its own pins:\n{out}"

    def one(job):
        tag, src, pin_file, expr, name = job
        lib = _build(str(tmp_path), tag, src)
        rc, out = _run_pins(lib, pin_file, expr)
        return name, rc, out

    workers = max(1, min(8, os.cpu_count() or 1))
    with ThreadPoolExecutor(workers) as ex:
        results = list(ex.map(one, jobs))
    # exit status 1: tests ran and at least one failed (anything else would
    # be a harness problem: nothing collected, an internal error)
    survivors = [(n, rc, out) for n, rc, out in results if rc != 1]
    assert not survivors, "slips not caught:\n" + "\n".join(
        f"- {n} (exit {rc})\n{out}" for n, rc, out in survivors)
