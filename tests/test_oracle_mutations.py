"""The pins catch plausible mistakes in the CPU reference.

Each case copies fpic_oracle.c, plants one mistake (a dropped term, a wrong
sign, a wrong index, a transposed operand, a wrong coefficient), builds the
copy and runs the pin suites against it in a subprocess: at least one pin
must fail.  Everything here runs on the CPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "fpic_oracle.c")

MUTANTS = {
    "commutator_sign": ("out[i][j] = -I * (Hr[i][j] - rH[i][j]);",
                        "out[i][j] = I * (Hr[i][j] - rH[i][j]);"),
    "antinu_vacuum_not_conjugated": ("Hb[i][j] = conj(Hv[i][j]) - conj(Hnn[i][j]);",
                                     "Hb[i][j] = Hv[i][j] - conj(Hnn[i][j]);"),
    "antinu_selfint_sign": ("Hb[i][j] = conj(Hv[i][j]) - conj(Hnn[i][j]);",
                            "Hb[i][j] = conj(Hv[i][j]) + conj(Hnn[i][j]);"),
    "flux_term_sign": ("h -= v[a] * (m->f[a][i][j] - conj(m->fb[a][i][j]));",
                       "h += v[a] * (m->f[a][i][j] - conj(m->fb[a][i][j]));"),
    "flux_term_dropped": ("h -= v[a] * (m->f[a][i][j] - conj(m->fb[a][i][j]));",
                          "(void)a;"),
    "nbar_not_conjugated": ("cplx h = m->n[i][j] - conj(m->nb[i][j]);",
                            "cplx h = m->n[i][j] - m->nb[i][j];"),
    "matmul_transposed": ("s += a[i][k] * b[k][j];", "s += a[k][i] * b[k][j];"),
    "cic_weights_swapped": ("w[0] = 1.0 - phi;\n    w[1] = phi;",
                            "w[0] = phi;\n    w[1] = 1.0 - phi;"),
    "quadratic_nearest_centre": ("const int up = phi < 0.5 ? 0 : 1;",
                                 "const int up = phi < 0.5 ? 1 : 0;"),
    "quadratic_centre_weight": ("w[1] = 0.75 - xi * xi;", "w[1] = 0.75 + xi * xi;"),
    "quadratic_edge_weights_swapped": ("w[0] = 0.5 * ((0.5 - xi) * (0.5 - xi));",
                                       "w[0] = 0.5 * ((0.5 + xi) * (0.5 + xi));"),
    "flux_wrong_axis": ("g->f[a][i][j] += wN * rho[i][j] * v[a];",
                        "g->f[a][i][j] += wN * rho[i][j] * v[2];"),
    "advection_backwards": ("left = pmod(home[a] + (int64_t)fl, P->ncell[a]);",
                            "left = pmod(home[a] - (int64_t)fl, P->ncell[a]);"),
    "rk4_k2_weight": ("ks[i] = ks[i] + 2.0 * k[i];\n            ys[i] = state[i] + (0.5 * dt) * k[i];",
                      "ks[i] = ks[i] + k[i];\n            ys[i] = state[i] + (0.5 * dt) * k[i];"),
    "rk4_stage_time": ("rhs(P, ys, stage_time(n, dt, 1.0), grid, k);",
                       "rhs(P, ys, stage_time(n, dt, 0.5), grid, k);"),
    "volume_not_divided": ("g->n[i][j] /= dV;", "g->n[i][j] /= 1.0;"),
    "gather_weight_dropped": ("out->n[i][j] += w * g->n[i][j];",
                              "out->n[i][j] += g->n[i][j];"),
    "matter_sign": ("H[a][a] += Vm[a];", "H[a][a] -= Vm[a];"),
    # general placement
    "general_cell_centre_offset": ("u = x / P->dx[a] - 0.5;", "u = x / P->dx[a];"),
    "general_drift_sign": ("const double x = P->pos0[3 * p + a] + P->pdirs[3 * p + a] * t;",
                           "const double x = P->pos0[3 * p + a] - P->pdirs[3 * p + a] * t;"),
    "general_nbar_weight": ("return P->pos0 ? P->pNbar[p] : P->Nbar[p / ncell_total(P)];",
                            "return P->pos0 ? P->pN[p] : P->Nbar[p / ncell_total(P)];"),
    "antinu_matter_sign": ("Hb[a][a] -= Vm[a];", "Hb[a][a] += Vm[a];"),
    # reverse mode
    "adjoint_rho_cotangent_sign": ("commutator_rhs(Gc, H, Xr);", "commutator_rhs(H, Gc, Xr);"),
    "adjoint_hbar_not_conjugated": ("Xn[i][j] = Xh[i][j] - conj(Xhb[i][j]);",
                                    "Xn[i][j] = Xh[i][j] - Xhb[i][j];"),
    "adjoint_flux_transpose_sign": ("q->f[a][i][j] -= w * v[a] * Xn[i][j];",
                                    "q->f[a][i][j] += w * v[a] * Xn[i][j];"),
    "adjoint_volume_dropped": ("Z[i][j] += w * zn / dV;", "Z[i][j] += w * zn;"),
    "adjoint_stage_coefficient": ("gs[i] = (dt / 3.0) * lam[i] + (0.5 * dt) * ls[i];",
                                  "gs[i] = (dt / 6.0) * lam[i] + (0.5 * dt) * ls[i];"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new))
    lib = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fopenmp", "-std=c11",
                    "-shared", "-fPIC", "-o", str(lib), str(mut), "-lm"],
                   check=True, capture_output=True)
    env = dict(os.environ, FPIC_ORACLE_LIB=str(lib), OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q",
                        "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_invariants.py"),
                        os.path.join(ROOT, "tests", "test_oracle_adjoint.py"),
                        os.path.join(ROOT, "tests", "test_oracle_particles.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=600)
    assert r.returncode != 0, f"no pin caught mutant {name}:\n{r.stdout[-2000:]}"
