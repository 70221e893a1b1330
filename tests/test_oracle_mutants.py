"""Planted mistakes: each test compiles a copy of the oracle with one plausible
error (a dropped term, a wrong sign or index, a transposed operand) and checks
that at least one pin of ``test_oracle`` fails against it.  Every mutant stays
inside its arrays, so a caught mistake is an assertion, never a crash."""
import os

import pytest

import oracle as orc
import test_oracle as pins
import test_oracle_mg as mg
import test_oracle_sell as sell

SRC = os.path.join(os.path.dirname(orc.__file__), "oracle.c")

# (name, original text, mutated text, pins that must catch it)
MUTANTS = [
    ("coo_transposed_operand",
     "y[ai[k]] += av[k] * x[aj[k]];\n}\n\n/* Algorithm 1 with float",
     "y[ai[k]] += av[k] * x[ai[k]];\n}\n\n/* Algorithm 1 with float",
     [lambda: pins.test_spmv_integer_bruteforce((7, 3), 0.6)]),
    ("coo_no_clear",
     "        y[i] = 0.0;\n    for (int64_t k = 0; k < nnz; ++k)\n        y[ai[k]] += av[k] * x[aj[k]];",
     "        y[i] = y[i];\n    for (int64_t k = 0; k < nnz; ++k)\n        y[ai[k]] += av[k] * x[aj[k]];",
     [pins.test_coo_spmv_overwrites_y_and_empty_rows_are_zero]),
    ("csr_wrong_column",
     "sum += av[j] * x[aj[j]];",
     "sum += av[j] * x[aj[j] > 0 ? aj[j] - 1 : 0];",
     [lambda: pins.test_spmv_integer_bruteforce((17, 17), 0.6)]),
    ("dia_bound_nrows",
     "if (k >= 0 && k < ncols)\n                sum += av[j * nrows + i] * x[k];",
     "if (k >= 0 && k < nrows)\n                sum += av[j * nrows + i] * x[k];",
     [pins.test_dia_bound_uses_ncols_for_rectangular]),
    ("dia_row_major_layout",
     "sum += av[j * nrows + i] * x[k];",
     "sum += av[i * ndiag + j] * x[k];",
     [lambda: pins.test_stencil_integer_x_all_formats_bit_identical(7)]),
    ("csr_pointer_shift",
     "irp[ai[k] + 1]++;",
     "irp[ai[k]]++;",
     [lambda: pins.test_stencil_csr_and_dia_closed_forms(4)]),
    ("dia_offset_sign",
     "doff[nd++] = (int32_t)(s - (nrows - 1));",
     "doff[nd++] = (int32_t)((nrows - 1) - s);",
     [lambda: pins.test_stencil_csr_and_dia_closed_forms(4)]),
    ("cg_residual_sign",
     "r[i] -= alpha * q[i];\n            rho_new",
     "r[i] += alpha * q[i];\n            rho_new",
     [lambda: pins.test_cg_small_spd_matches_solve(12, 2)]),
    ("cg_beta_inverted",
     "double beta = rho_new / rho;",
     "double beta = rho / rho_new;",
     [lambda: pins.test_cg_small_spd_matches_solve(30, 3)]),
    ("cg_no_direction_update",
     "p[i] = r[i] + beta * p[i];\n            rho = rho_new;",
     "p[i] = r[i] + 0.0 * beta * p[i];\n            rho = rho_new;",
     [pins.test_cg_diagonal_distinct_eigenvalues_iteration_count,
      lambda: pins.test_cg_stencil_recovers_ones_within_kappa_bound(8, 1e-9)]),
    ("mixed_missing_scale",
     "x[i] += rn * (double)d[i];",
     "x[i] += (double)d[i];",
     [lambda: pins.test_mixed_refinement_reaches_fp64_residual(8)]),
    ("ru_update_drops_correction",
     "                x[i] += (double)d[i];\n                d[i] = 0.0f;",
     "                x[i] += 0.0 * (double)d[i];\n                d[i] = 0.0f;",
     [lambda: pins.test_reliable_update_reaches_fp64_residual(5, 0.1)]),
    ("ru_keeps_fp32_residual",
     "            for (int64_t i = 0; i < n; ++i)\n                r32[i] = (float)r[i];\n            rho_new",
     "            for (int64_t i = 0; i < n; ++i)\n                r32[i] = r32[i];\n            rho_new",
     [pins.test_reliable_update_on_spd_matches_solve]),
    ("ru_alpha_inverted",
     "            break;\n        }\n        float alpha = (float)(rho / sigma);",
     "            break;\n        }\n        float alpha = (float)(sigma / rho);",
     [pins.test_reliable_update_first_iterate]),
    ("split_strict_threshold",
     "if (count[s] > 0 && (double)count[s] >= min_fill * (double)slots)",
     "if (count[s] > 0 && (double)count[s] > min_fill * (double)slots)",
     [pins.test_split_band_hand_built]),
    ("split_slots_square_only",
     "int64_t hi = ncols - d < nrows ? ncols - d : nrows;",
     "int64_t hi = nrows - d < nrows ? nrows - d : nrows;",
     [pins.test_split_band_full_rectangular_and_stencil]),
    ("features_variance_not_normalised",
     "var = nrows ? var / (double)nrows : 0.0;",
     "var = var;",
     [lambda: pins.test_features_stencil_closed_form(5)]),
    ("mlp_relu_derivative_dropped",
     "dh2[k] = a2[k] > 0.0 ? g : 0.0;",
     "dh2[k] = g;",
     [pins.test_mlp_gradient_matches_finite_differences]),
    ("mlp_w2_transposed",
     "s += h1[j] * w[OFF_W2 + j * NH + k];",
     "s += h1[j] * w[OFF_W2 + k * NH + j];",
     [pins.test_mlp_gradient_matches_finite_differences]),
    ("symgs_backward_runs_forward",
     "    for (int64_t t = n - 1; t >= 0; --t)\n        if (gs_row(irp, aj, av, order[t], r, x) != ORC_OK)",
     "    for (int64_t t = 0; t < n; ++t)\n        if (gs_row(irp, aj, av, order[t], r, x) != ORC_OK)",
     [lambda: mg.test_gs_sweeps_are_triangular_solves("stencil5", "natural")]),
    ("gs_diagonal_also_subtracted",
     "        if (aj[k] == i)\n            d = av[k];\n        else\n            s -= av[k] * x[aj[k]];",
     "        if (aj[k] == i)\n            d = av[k];\n        s -= av[k] * x[aj[k]];",
     [lambda: mg.test_gs_sweeps_are_triangular_solves("random60", "permuted")]),
    ("ell_row_major",
     "irp[i];\n            ecol[k * nrows + i] = k < len ? aj[irp[i] + k] : -1;\n            eval[k * nrows + i] = k < len ? av[irp[i] + k] : 0.0;",
     "irp[i];\n            ecol[i * K + k] = k < len ? aj[irp[i] + k] : -1;\n            eval[i * K + k] = k < len ? av[irp[i] + k] : 0.0;",
     [sell.test_ell_hand_built_layout]),
    ("sell_sorted_ascending",
     "for (int64_t len = maxlen; len >= 0; --len)",
     "for (int64_t len = 0; len <= maxlen; ++len)",
     [lambda: sell.test_sell_perm_sorts_windows_stably(64)]),
    ("sell_width_of_first_row",
     "            if (len > w)\n                w = len;\n        }\n        cs[s + 1]",
     "            if (p == s * C)\n                w = len;\n        }\n        cs[s + 1]",
     [lambda: sell.test_spmv_integer_bruteforce(4, 1, (17, 17), 0.3),
      lambda: sell.test_sell_perm_sorts_windows_stably(1)]),
    ("sell_result_unpermuted",
     "        y[perm[p]] = sum;",
     "        y[p] = sum;",
     [lambda: sell.test_spmv_integer_bruteforce(4, 8, (17, 17), 0.3)]),
    ("hyb_no_row_floor",
     "int64_t need = nrows / 3 > 4096 ? nrows / 3 : 4096;",
     "int64_t need = nrows / 3;",
     [sell.test_hyb_width_rule_hand_built]),
    ("hyb_rest_skips_an_entry",
     "        for (int64_t k = K; k < len; ++k) {\n            ri[q]",
     "        for (int64_t k = K + 1; k < len; ++k) {\n            ri[q]",
     [lambda: sell.test_hyb_partition_and_spmv("random37x53", sell.CASES[1][1], 1)]),
    ("adam_no_bias_correction",
     "double mh = m[i] / c1, vh = v[i] / c2;",
     "double mh = m[i], vh = v[i];",
     [pins.test_adam_first_step_is_signed_lr]),
]


@pytest.mark.parametrize("name,old,new,catchers", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new, catchers):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mutant_src = tmp_path / f"{name}.c"
    mutant_src.write_text(src.replace(old, new))
    lib = orc.build(out=str(tmp_path / f"{name}.so"), src=str(mutant_src))
    caught = 0
    with orc.use_library(lib):
        for pin in catchers:
            try:
                pin()
            except AssertionError:
                caught += 1
    assert caught >= 1, f"no pin caught the planted mistake {name}"


# Mistakes in the Python part of the oracle (the V-cycle and PCG): a copy of
# the module with one edit, run through the pins that take the module.
PY_MUTANTS = [
    ("coarse_point_odd",
     "return (2 * ci + 2 * cj * n + 2 * ck * n * n).astype(np.int64)",
     "return (2 * ci + 1 + 2 * cj * n + 2 * ck * n * n).astype(np.int64)",
     [lambda m: mg.test_coarse_points_are_even_coordinates(4, m=m),
      lambda m: mg.test_vcycle_two_levels_by_library_solves(4, m=m)]),
    ("restriction_drops_Az",
     "zc = cycle(l + 1, rl[f] - az[f])",
     "zc = cycle(l + 1, rl[f])",
     [lambda m: mg.test_vcycle_two_levels_by_library_solves(8, m=m)]),
    ("prolongation_sign",
     "z[f] += zc",
     "z[f] -= zc",
     [lambda m: mg.test_vcycle_two_levels_by_library_solves(8, m=m)]),
    ("no_post_smoothing",
     "        z[f] += zc\n        st, z = symgs(irp, aj, av, orders[l], rl, z)",
     "        z[f] += zc",
     [lambda m: mg.test_vcycle_symmetric_positive(8, 2, m=m)]),
    ("pcg_beta_inverted",
     "p = z.copy() if k == 0 else z + (rz / rz_old) * p",
     "p = z.copy() if k == 0 else z + (rz_old / rz) * p",
     [lambda m: mg.test_pcg_identity_preconditioner_is_cg(6, m=m)]),
    ("pcg_alpha_from_rr",
     "alpha = rz / sigma",
     "alpha = dot(r, r) / sigma",
     [lambda m: mg.test_pcg_with_vcycle_converges_faster_and_to_ones(m=m)]),
]


@pytest.mark.parametrize("name,old,new,catchers", PY_MUTANTS, ids=[m[0] for m in PY_MUTANTS])
def test_planted_python_mistake_is_caught(tmp_path, name, old, new, catchers):
    import importlib.util
    path = os.path.join(os.path.dirname(orc.__file__), "__init__.py")
    src = open(path).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    # the copy keeps using the real oracle library
    src = src.replace("_HERE = os.path.dirname(os.path.abspath(__file__))",
                      f"_HERE = {os.path.dirname(path)!r}")
    mpath = tmp_path / f"{name}.py"
    mpath.write_text(src.replace(old, new))
    spec = importlib.util.spec_from_file_location(f"oracle_mutant_{name}", mpath)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    caught = 0
    for pin in catchers:
        try:
            pin(mod)
        except AssertionError:
            caught += 1
    assert caught >= 1, f"no pin caught the planted mistake {name}"
