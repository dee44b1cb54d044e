"""The oracle's pins must catch plausible mistakes.  Each case plants one
mistake (a dropped term, a wrong sign, a transposed operand, a wrong index)
in a copy of the C oracle, builds it on the CPU, swaps it in, and checks that
at least one pin fails.  CPU only; nothing here touches the HIP library."""
import ctypes
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle
import tests.test_oracle_adjoint as t_adj
import tests.test_oracle_geometry as t_geo
import tests.test_oracle_gs as t_gs
import tests.test_oracle_operator as t_op
import tests.test_oracle_reference_element as t_ref
import tests.test_oracle_solve as t_sol

SRC = os.path.join(os.path.dirname(oracle.__file__), "sem_oracle.c")

# (name, original text, mutated text)
MUTANTS = [
    ("legendre_recurrence_coeff", "double dk = dm2 + (2.0 * k - 1.0) * pm1;",
     "double dk = dm2 + (2.0 * k + 1.0) * pm1;"),
    ("gll_weight_power", "rho[j] = 2.0 / (N * (N + 1.0) * p * p);",
     "rho[j] = 2.0 / (N * (N + 1.0) * fabs(p));"),
    ("dhat_diag_sign", "D[i * nq + i] = -s;", "D[i * nq + i] = s;"),
    ("dhat_offdiag_transposed", "D[i * nq + l] = pn[i] / (pn[l] * (xi[i] - xi[l]));",
     "D[i * nq + l] = pn[l] / (pn[i] * (xi[i] - xi[l]));"),
    ("geom_ds_index", "ds += D[j * nq + l] * X[p][IDX(i, l, k, e)];",
     "ds += D[l * nq + j] * X[p][IDX(i, l, k, e)];"),
    ("geom_cofactor_sign", "R[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) / det;",
     "R[0][1] = (M[0][1] * M[2][2] - M[0][2] * M[2][1]) / det;"),
    ("geom_metric_transposed", "for (int l = 0; l < 3; ++l) s += R[m][l] * R[mp][l];",
     "for (int l = 0; l < 3; ++l) s += R[l][m] * R[l][mp];"),
    ("geom_mass_weight", "double b = rho[i] * rho[j] * rho[k] * det;",
     "double b = rho[i] * rho[j] * rho[i] * det;"),
    ("ax_transposed_DT", "s += D[l * nq + i] * wr[l + nq * (j + nq * k)];",
     "s += D[i * nq + l] * wr[l + nq * (j + nq * k)];"),
    ("ax_dropped_t_term", "s += D[l * nq + k] * wt[i + nq * (j + nq * l)];", "(void)0;"),
    ("ax_wrong_G_entry", "ws[lq] = c * (g12 * ur + g22 * us + g23 * ut);",
     "ws[lq] = c * (g12 * ur + g22 * us + g13 * ut);"),
    ("ax_helmholtz_sign", "if (h2 != 0.0) v += h2 * B[q] * u[q];",
     "if (h2 != 0.0) v -= h2 * B[q] * u[q];"),
    ("diag_cross_factor", "s += 2.0 * di * dj * KG(1, q) + 2.0 * di * dk * KG(2, q)",
     "s += di * dj * KG(1, q) + 2.0 * di * dk * KG(2, q)"),
    ("qqt_drop_writeback_first", "if (cid[l] >= 0) v[l] = acc[cid[l]];",
     "if (cid[l] >= 0 && l > 0) v[l] = acc[cid[l]];"),
    ("maps_keep_singles", "if (b - a >= 2) {", "if (b - a >= 1) {"),
    ("gradk_sign", "gk[q] = -h1 * s;", "gk[q] = h1 * s;"),
    ("gradk_wrong_u_index", "c[1] += D[j * nq + l] * u[IDX(i, l, k, e)];",
     "c[1] += D[j * nq + l] * u[IDX(l, i, k, e)];"),
    ("interp_wrong_node", "if (m != j) h *= (xt[i] - xs[m]) / (xs[j] - xs[m]);",
     "if (m != j) h *= (xt[i] - xs[m]) / (xs[i % ns] - xs[m] + (i % ns == m));"),
    ("interp_lvec_axes_swapped", "s += J[k * ns + c] * J[j * ns + b] * J[i * ns + a]",
     "s += J[j * ns + c] * J[k * ns + b] * J[i * ns + a]"),
    ("interp_lvec_transposed_J", "s += J[k * ns + c] * J[j * ns + b] * J[i * ns + a]",
     "s += J[k * ns + c] * J[j * ns + b] * J[a * nt + i]"),
    ("interp_lvec_element_stride", "* in[e * pin + a + ns * (b + ns * c)];",
     "* in[e * pout % (pin * E) + a + ns * (b + ns * c)];"),
    ("gsop_min_as_max", "acc[c] = fmin(acc[c], v[l]);", "acc[c] = fmax(acc[c], v[l]);"),
    ("gsop_first_copy_dropped", "acc[c] = v[l];\n            seen[c] = 1;", "acc[c] = 1.0;\n            seen[c] = 1;"),
    ("gsop_mul_as_add", "acc[c] = acc[c] * v[l];", "acc[c] = acc[c] + v[l];"),
]

PINS = [
    t_ref.test_gll_closed_forms,
    lambda gd: t_ref.test_gll_against_library_roots_and_sums(5),
    lambda gd: t_ref.test_dhat_differentiates_polynomials_exactly(5),
    lambda gd: t_ref.test_dhat_known_entries(3),
    lambda gd: t_ref.test_interp_matrix(),
    lambda gd: t_ref.test_interp_lvec_reproduces_polynomials(7, 3),
    lambda gd: t_ref.test_interp_lvec_reproduces_polynomials(2, 5),
    lambda gd: t_geo.test_undeformed_cube_closed_form(3),
    lambda gd: t_geo.test_affine_nonsymmetric_map(),
    lambda gd: t_geo.test_deformed_volume_converges_spectrally(),
    lambda gd: t_op.test_ax_equals_dense_kronecker((2, 1, 1), 3),
    lambda gd: t_op.test_undeformed_element_closed_form(3),
    lambda gd: t_op.test_energy_of_polynomial_on_box(4),
    lambda gd: t_op.test_assembled_operator_properties(2),
    lambda gd: t_gs.test_multiplicity_and_maps((3, 2, 1), 3),
    lambda gd: t_gs.test_qqt_dense_and_contract(),
    lambda gd: t_gs.test_qqt_sums_in_ascending_local_order(),
    lambda gd: t_gs.test_gs_op_brute_force_and_invariants("mul"),
    lambda gd: t_gs.test_gs_op_brute_force_and_invariants("min"),
    lambda gd: t_gs.test_gs_op_order_and_closed_forms(),
    lambda gd: t_sol.test_pcg_matches_dense_cholesky(0.0),
    lambda gd: t_adj.test_adjoint_gradients_vs_central_differences(),
]


def _build(src_text, d):
    c = os.path.join(d, "m.c")
    so = os.path.join(d, "m.so")
    with open(c, "w") as fh:
        fh.write(src_text)
    subprocess.check_call(["gcc", "-std=gnu11", "-O1", "-fPIC", "-shared", c, "-o", so, "-lm"])
    return so


def _swap_in(so):
    L = ctypes.CDLL(so)
    ref = oracle.lib()
    for fn in ("oracle_gll", "oracle_dhat", "oracle_interp", "oracle_geometry", "oracle_ax",
               "oracle_diag", "oracle_qqt", "oracle_gs_op", "oracle_multiplicity", "oracle_gs_maps",
               "oracle_grad_k", "oracle_interp_lvec"):
        getattr(L, fn).argtypes = getattr(ref, fn).argtypes
    return L


def _run_pins(so, golden_dir):
    saved = oracle.lib()
    oracle._lib = _swap_in(so)
    failed = []
    try:
        for i, pin in enumerate(PINS):
            try:
                pin(golden_dir)
            except Exception as exc:  # any pin failure counts
                failed.append((i, type(exc).__name__))
                break
    finally:
        oracle._lib = saved
    return failed


def test_control_unmutated_copy_passes_every_pin(golden_dir):
    d = tempfile.mkdtemp()
    try:
        so = _build(open(SRC).read(), d)
        assert _run_pins(so, golden_dir) == []
    finally:
        shutil.rmtree(d, ignore_errors=True)


@pytest.mark.parametrize("name,orig,mut", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_catch_mutant(name, orig, mut, golden_dir):
    src = open(SRC).read()
    assert src.count(orig) == 1, f"mutation anchor for {name} not found exactly once"
    d = tempfile.mkdtemp()
    try:
        so = _build(src.replace(orig, mut), d)
        assert _run_pins(so, golden_dir), f"no pin caught mutant {name}"
    finally:
        shutil.rmtree(d, ignore_errors=True)
