"""Planted mistakes in a copy of the oracle must be caught by the pins.

Each mutation edits the oracle's C source text (a transposed operand, a
dropped term, a wrong index, a swapped factor, a flipped sign), builds the
altered copy into a temporary library on the CPU, and runs every pin against
it in a child process.  A mutation that no pin catches fails this test.  The
real oracle is never modified.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "kron_oracle.c")

MUTATIONS = {
    "2d_B_transposed": ("B[r + n * l] * x[l + n * m]", "B[l + n * r] * x[l + n * m]"),
    "2d_A_not_transposed": ("tmp[r + n * m] * A[c + n * m]", "tmp[r + n * m] * A[m + n * c]"),
    "2d_X_transposed": ("B[r + n * l] * x[l + n * m]", "B[r + n * l] * x[m + n * l]"),
    "2d_dropped_term": ("for (int l = 0; l < n; ++l) s += B[r + n * l]", "for (int l = 1; l < n; ++l) s += B[r + n * l]"),
    "2d_output_transposed": ("y[r + n * c] = s;", "y[c + n * r] = s;"),
    "3d_factor_order": ("KPQR(n, C, B, A, X + p * nnn", "KPQR(n, A, B, C, X + p * nnn"),
    "3d_P_transposed": ("s += P[i + n * l] * x", "s += P[l + n * i] * x"),
    "3d_Q_transposed": ("s += Q[j + n * m] * w1", "s += Q[m + n * j] * w1"),
    "3d_R_transposed": ("s += R[k + n * q] * w2", "s += R[q + n * k] * w2"),
    "3d_dropped_term": ("for (int m = 0; m < n; ++m) s += Q", "for (int m = 0; m + 1 < n; ++m) s += Q"),
    "3d_wrong_slab": ("w2[i + n * j + nn * q] = s;", "w2[j + n * i + nn * q] = s;"),
    "3d_output_stride": ("Y + p * nnn, w1, w2", "Y + p * nnn - (p > 0 ? 1 : 0), w1, w2"),
    "grad2d_dX_untransposed": ("oracle_kron2d_f64(n, At, Bt, dY, dX, batch)", "oracle_kron2d_f64(n, A, B, dY, dX, batch)"),
    "grad2d_dA_index": ("dA[c + n * m] += s;", "dA[m + n * c] += s;"),
    "grad2d_dB_sign": ("dB[r + n * l] += s;", "dB[r + n * l] -= s;"),
    "grad2d_dB_missing_A": ("s += x[l + n * m] * A[c + n * m]", "s += x[l + n * m] * A[m + n * c]"),
    "grad3d_dX_untransposed": ("oracle_kron3d_f64(n, At, Bt, Ct, dY, dX, batch)", "oracle_kron3d_f64(n, At, Bt, C, dY, dX, batch)"),
    "grad3d_U_factors": ("kpqr_f64(n, C, B, I, x, u, w1, w2);", "kpqr_f64(n, B, C, I, x, u, w1, w2);"),
    "grad3d_dB_index": ("dB[j + n * b] += s;", "dB[b + n * j] += s;"),
    "grad3d_dC_contraction": ("u[i * nn + j * n + c];", "u[i * nn + c * n + j];"),
    "ex_transpose_ignored": ("const int t = (op == 'T' || op == 't');", "const int t = 0;"),
    "ex_alpha_dropped": ("y[e] = beta == 0.0 ? alpha * z[e] : alpha * z[e] + beta * y[e];",
                         "y[e] = beta == 0.0 ? z[e] : z[e] + beta * y[e];"),
    "ex_beta_zero_reads_y": ("y[e] = beta == 0.0 ? alpha * z[e] : alpha * z[e] + beta * y[e];",
                             "y[e] = alpha * z[e] + beta * y[e];"),
    "ex_ops_swapped": ("  op_matrix(n, opA, A, Ao);\n  op_matrix(n, opB, B, Bo);\n  op_matrix(n, opC, C, Co);",
                       "  op_matrix(n, opB, A, Ao);\n  op_matrix(n, opA, B, Bo);\n  op_matrix(n, opC, C, Co);"),
    "ex_op_x_ignored": ("op_matrix(n, opX, X + p * nn, xo + p * nn);", "op_matrix(n, 'N', X + p * nn, xo + p * nn);"),
    "tkron1_transpose_ignored": ("  op_matrix(n, opA, A, Ao);\n  for (int64_t p = 0; p < batch; ++p) {\n    const double* x = X + p * ldxp;",
                                 "  op_matrix(n, 'N', A, Ao);\n  for (int64_t p = 0; p < batch; ++p) {\n    const double* x = X + p * ldxp;"),
    "tkron1_output_stride": ("    double* y = Y + p * ldyp;", "    double* y = Y + p * ldxp;"),
    "nd_op_n_transposed": ("((op) == 'N' || (op) == 'n' ? (M)[(i) + (int64_t)(ld) * (a)]",
                           "((op) == 'N' || (op) == 'n' ? (M)[(a) + (int64_t)(ld) * (i)]"),
    "nd_conj_dropped": ("DEFINE_KRON_ND(kron_nd_cplx, double _Complex, conj)",
                        "DEFINE_KRON_ND(kron_nd_cplx, double _Complex, ND_NO_CONJ)"),
    "nd_per_operand_factor_ignored": ("const T* M = F[k] + p * ldfp[k];", "const T* M = F[k];"),
    "nd_dropped_term": ("for (int a = 0; a < n[k]; ++a)", "for (int a = 1; a < n[k]; ++a)"),
    "nd_alpha_dropped": ("T v = alpha * cur[q];", "T v = cur[q];"),
    "nd_beta_zero_reads_y": ("Y[p * ny + q] = beta == (T)0 ? v : v + beta * Y[p * ny + q];",
                             "Y[p * ny + q] = v + beta * Y[p * ny + q];"),
    "nd_wrong_post_index": ("cur[(u * n[k] + a) * post + v];", "cur[(u * n[k] + a) * post + (post - 1 - v)];"),
    "nd_output_row_index": ("nxt[(u * m[k] + i) * post + v] = s;", "nxt[(u * m[k] + (m[k] - 1 - i)) * post + v] = s;"),
    "f32_accumulates_in_double": ("DEFINE_KRON2D(oracle_kron2d_f32, float)", "DEFINE_KRON2D(oracle_kron2d_f32_unused, float)\nORACLE_API void oracle_kron2d_f32(int n, const float* A, const float* B, const float* X, float* Y, int64_t batch) { (void)A; (void)B; for (int64_t i = 0; i < batch * n * n; ++i) Y[i] = X[i]; }"),
}

RUNNER = r"""
import sys
sys.path.insert(0, {root!r}); sys.path.insert(0, {tests!r})
import oracle, pins
orc = oracle.Oracle({lib!r})
caught = []
for pin in pins.ALL_PINS:
    try:
        pin(orc)
    except AssertionError:
        caught.append(pin.__name__)
print("CAUGHT", ",".join(caught))
"""


def _run_pins_on(source_text):
    with tempfile.TemporaryDirectory() as td:
        src = os.path.join(td, "kron_oracle.c")
        lib = os.path.join(td, "liboracle_mut.so")
        with open(src, "w") as f:
            f.write(source_text)
        subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                        "-ffp-contract=off", src, "-o", lib], check=True)
        code = RUNNER.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
        r = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, timeout=300)
    caught = r.stdout.split("CAUGHT", 1)[1].strip() if "CAUGHT" in r.stdout else None
    return r, caught


def test_unaltered_copy_passes_every_pin():
    r, caught = _run_pins_on(open(SRC).read())
    assert r.returncode == 0 and caught == "", (r.stdout, r.stderr[-800:])


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name):
    old, new = MUTATIONS[name]
    text = open(SRC).read()
    assert text.count(old) >= 1, f"mutation anchor for {name} not found in the oracle source"
    r, caught = _run_pins_on(text.replace(old, new, 1))
    # caught by a pin, or the altered oracle crashed (killed by a signal)
    assert (r.returncode == 0 and caught) or r.returncode < 0, \
        f"no pin caught mutation {name}: rc={r.returncode} {r.stdout} {r.stderr[-500:]}"
