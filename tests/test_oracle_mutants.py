"""Plausible mistakes planted in copies of the oracle must each trip a pin.

Every mutant is a textual edit of ``oracle/lagp_oracle.c`` compiled into a
temporary directory; the real oracle is never modified.
"""
import pytest

import oracle
import oracle_pins

MUTANTS = {
    # batch scores: covariance sign flipped, and the nugget left off K_j
    "scores_cov_sign": ("const double cov = kcx - dot(z, zh, j);", "const double cov = kcx + dot(z, zh, j);"),
    "scores_no_nugget": ("        K[a * j + a] += g;\n        hv[a]", "        K[a * j + a] += 1e-9;\n        hv[a]"),
    # the sign slip of Fig. 3 step 5 taken literally: (c + u.h)^2 / s
    "cov_sign": ("double cov = kcx - dot(w->zc, w->zh, j);", "double cov = kcx + dot(w->zc, w->zh, j);"),
    # nugget dropped from the candidate self-covariance
    "kappa_no_nugget": ("    const double kappa = 1.0 + g;\n    for (int k = 0; k < p; k++)\n"
                        "        if (!isfinite(x[k])) return ORC_NONFINITE;\n    memset(w->chosen, 0, (size_t)Np);\n"
                        "    for (int q = 0; q < 5; q++) tr->pred",
                        "    const double kappa = 1.0;\n    for (int k = 0; k < p; k++)\n"
                        "        if (!isfinite(x[k])) return ORC_NONFINITE;\n    memset(w->chosen, 0, (size_t)Np);\n"
                        "    for (int q = 0; q < 5; q++) tr->pred"),
    # nugget wrongly added to the cross-covariance with x
    "nugget_on_h": ("w->h[a] = kern2(xa, x, p, d, dsep);", "w->h[a] = kern2(xa, x, p, d, dsep) + g;"),
    # transposed operand in the triangular solve
    "solve_transposed": ("for (int k = 0; k < r; k++) s -= L[r * j + k] * z[k];",
                         "for (int k = 0; k < r; k++) s -= L[k * j + r] * z[k];"),
    # score ties go to the largest index
    "tie_reversed": ("(delta == best && best_slot >= 0 && pool[s] < pool[best_slot])",
                     "(delta == best && best_slot >= 0 && pool[s] > pool[best_slot])"),
    # pool ties broken by descending index
    "pool_tie_reversed": ("return (a->idx > b->idx) - (a->idx < b->idx);",
                          "return (a->idx < b->idx) - (a->idx > b->idx);"),
    # Student-t scale divided by n - 1
    "s2_divisor": ("double s2 = psi * v / n;", "double s2 = psi * v / (n - 1);"),
    # psi = Y^T Y instead of Y^T K^{-1} Y
    "psi_wrong": ("double psi = dot(Yd, alpha, n);\n        double v = kappa",
                  "double psi = dot(Yd, Yd, n);\n        double v = kappa"),
    # NN start skips the nearest point
    "init_off_by_one": ("                take_slot = j;\n", "                take_slot = j + 1;\n"),
    # last coordinate dropped from the distance
    "dist_drops_coord": ("    for (int k = 0; k < p; k++) {\n        double t = a[k] - b[k];\n        s = s + t * t;\n",
                         "    for (int k = 0; k + 1 < p; k++) {\n        double t = a[k] - b[k];\n        s = s + t * t;\n"),
    # partitioned inverse with the sign of g flipped (mode B)
    "piedef_sign": ("for (int a = 0; a < j; a++) gv[a] = -m * u[a];\n    int J",
                    "for (int a = 0; a < j; a++) gv[a] = m * u[a];\n    int J"),
    # Cholesky diagonal without the square root
    "chol_no_sqrt": ("L[r * j + r] = sqrt(s);", "L[r * j + r] = s;"),
    # eq. gpk without its Gamma-function constant
    "nll_no_lgamma": ("double nll = -lgamma(0.5 * n) + 0.5 * n * log(2.0 * M_PI)",
                      "double nll = 0.5 * n * log(2.0 * M_PI)"),
    # derivative of K in d with the wrong power of d
    "kd_power": ("Kd[a * n + b] = c * r2 / (d * d);", "Kd[a * n + b] = c * r2 / d;"),
    # trace term without its factor 1/2
    "dd_trace_half": ("out[1] = 0.5 * trAKd - 0.5 * n * aKda / psi;", "out[1] = trAKd - 0.5 * n * aKda / psi;"),
    # nugget derivative with the wrong quadratic form
    "dg_form": ("out[2] = 0.5 * trA - 0.5 * n * aa / psi;", "out[2] = 0.5 * trA - 0.5 * n * aKda / psi;"),
    # second derivative missing the psi^2 term
    "d2_missing_term": ("+ aKda * aKda / (psi * psi));", ");"),
    # mode-B prediction: mean from Y instead of K(X_n, x)
    "pred_b_mean": ("                mu += w->h[a] * alpha_a;", "                mu += w->Yn[a] * alpha_a;"),
    # fixed-design mode-B prediction: variance term with the wrong vector
    "predict_b_hwh": ("hwh += h[a] * dot(A + (size_t)a * n, h, n);", "hwh += h[a] * dot(A + (size_t)a * n, Yd, n);"),
    # psi trajectory from Y_j^T Y_j
    "psitraj_plain": ("tr->psitraj[j] = j > 0 ? dot(w->ty, w->ty, j) : 0.0;",
                      "tr->psitraj[j] = j > 0 ? dot(w->yj, w->yj, j) : 0.0;"),
    # batched MLE gathering the first location's responses for every design
    "local_mle_gather": ("Yn[a] = Y[sel[m * n + a]];", "Yn[a] = Y[sel[a]];"),
    # MSPE: expected information without the unknown scale's share
    "mspe_info_no_scale": ("G = 0.5 * (tW2 - tW * tW / J1);", "G = 0.5 * tW2;"),
    # MSPE: mean derivative without the K^{-1} Kdot K^{-1} term
    "mspe_dmu_one_term": ("const double dm = hd_al - w_kd_al;", "const double dm = hd_al;"),
    # MSPE: variance factor (j + 1) psi / (j (j - 1)) with j - 1 replaced by j
    "mspe_coef": ("const double coef = (j + 1) * psi / ((double)j * (j - 1));",
                  "const double coef = (j + 1) * psi / ((double)j * j);"),
    # MSPE: the largest criterion chosen instead of the smallest
    "mspe_argmax": ("if (crit < best || (crit == best && best_slot >= 0 && pool[s] < pool[best_slot])) {",
                    "if (!(crit <= best) || best_slot < 0 || (crit == best && pool[s] < pool[best_slot])) {"),
    # separable kernel: lengthscales paired with the wrong inputs
    "sep_index_shift": ("s = s + t * t / dsep[k];", "s = s + t * t / dsep[(k + 1) % p];"),
    # separable kernel: the location's kernel vector h left isotropic
    "sep_h_isotropic": ("w->h[a] = kern2(xa, x, p, d, dsep);", "w->h[a] = kern(xa, x, p, d);"),
    # Newton iteration stopping on the first backtracking success without moving on
    "mle_one_step": ("        if (moved <= 1e-10 * d) { status = 0; it++; break; }",
                     "        status = 0; it++; break;"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(oracle.SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    path = tmp_path / f"{name}.c"
    path.write_text(src.replace(old, new))
    lib = oracle.compile_c(str(path), str(tmp_path / f"lib{name}.so"))
    orc = oracle.Oracle(lib)
    tripped = []
    for pin in oracle_pins.ALL:
        try:
            pin(orc)
        except Exception:  # any failure, including garbage indices, counts
            tripped.append(pin.__name__)
    assert tripped, f"mutant {name} passed every pin"
