"""The oracle's pins have teeth: each planted mistake below (a dropped term, a wrong
sign or index, a transposed operand) must make at least one pin fail.

Mistakes are planted in a private copy of the oracle's source on the CPU; the real
oracle is never modified.
"""
import importlib.util
import os
import shutil
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
TESTS = os.path.join(ROOT, "tests")

MUTATIONS = [
    # (file, original text, planted mistake)
    ("lupp.py", "prod = l[:, None] * T[p, t + 1:][None, :]",
     "prod = -l[:, None] * T[p, t + 1:][None, :]"),                      # sign of update
    ("lupp.py", "if rows.size and t + 1 < K:", "if False:"),              # dropped update
    ("lupp.py", "l = T[rows, t] / T[p, t]", "l = T[rows, t] / T[p, t + 1 if t + 1 < K else t]"),
    ("lupp.py", "p = int(np.argmax(mag))",
     "p = int(np.argmax(np.where(mag < 0, -1.0, mag ** 0.5 + np.arange(mag.size) * 1e-3)))"),
    ("icur.py", "S = X0 - (X0[:, J] @ U) @ A[I, :]",
     "S = X0 - (X0[:, J] @ U.T) @ A[I, :]"),                             # transposed operand
    ("icur.py", "Sr = A[:, Jk] - A[:, J] @ (U @ A[np.ix_(I, Jk)])",
     "Sr = A[:, Jk] + A[:, J] @ (U @ A[np.ix_(I, Jk)])"),                 # sign
    ("icur.py", "Ik, rm = pick(Sr, len(Jk), exclude=I, return_margins=True)",
     "Ik, rm = pick(A[:, Jk], len(Jk), exclude=I, return_margins=True)"),  # not the residual
    ("icur.py", "Jk, cm = pick(S.T, s, exclude=J, return_margins=True)",
     "Jk, cm = pick(X0.T, s, exclude=J, return_margins=True)"),    # sketch not downdated
    ("icur.py", "rho = np.linalg.norm(S) / denom", "rho = np.linalg.norm(S) / np.linalg.norm(A)"),
    ("icur.py", "X0 = G @ A", "X0 = G[:, ::-1] @ A"),                      # wrong index
    ("icur.py", "return (11 * int(b)) // 10", "return (11 * int(b) + 9) // 10"),
    ("rng.py", "for rnd in range(10):", "for rnd in range(9):"),
    ("rng.py", "np.uint64(0x7FFF) + ((bits", "np.uint64(0x8000) + ((bits"),
    ("rng.py", "x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(ka), lo1, hi0 ^ x3 ^ np.uint64(kb), lo0)",
     "x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(kb), lo1, hi0 ^ x3 ^ np.uint64(ka), lo0)"),
    ("rng.py", "rows[:, t] = np.where(taken, j, v)", "rows[:, t] = v"),   # Floyd step dropped
    # replay mode
    ("lupp.py", 'val = abs(T[p, t])', 'val = abs(T[b, t])'),             # value of the argmax
    # QRCP
    ("qrcp.py", "nrm = np.sqrt(np.sum(X[t:, :] ** 2, axis=0))",
     "nrm = np.sqrt(np.sum(X[:, :] ** 2, axis=0))"),                       # full, not trailing norms
    ("qrcp.py", "beta = 0.0 if vv == 0.0 else 2.0 / vv", "beta = 0.0 if vv == 0.0 else 1.0 / vv"),
    # SRTT operator and the sketch scale
    ("rng.py", "q = (rows[:, None] * (2 * i[None, :] + 1)) % (4 * m)",
     "q = (rows[:, None] * (2 * i[None, :] + 1)) % (2 * m)"),              # wrong period
    ("rng.py", "scale = np.where(rows == 0, np.sqrt(1.0 / m), np.sqrt(2.0 / m)) * np.sqrt(m / c)",
     "scale = np.where(rows == 0, np.sqrt(2.0 / m), np.sqrt(2.0 / m)) * np.sqrt(m / c)"),
    ("rng.py", "chosen.add(j if v in chosen else v)", "chosen.add(v)"),     # Floyd step dropped
    ("rng.py", "return float(np.sqrt(c))", "return float(c)"),              # Gaussian scale
    # the ||A||_F denominator
    ("icur.py", 'denom = g if denominator == "GA" else g_scale(kind, c, zeta) * np.linalg.norm(A)',
     'denom = g if denominator == "GA" else np.linalg.norm(A)'),
]


def _load(path, name):
    spec = importlib.util.spec_from_file_location(name, path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def _pins_pass(pkg_parent):
    """Run a fixed set of pin checks against the oracle package found under
    pkg_parent; return True when all of them pass."""
    saved = {k: v for k, v in sys.modules.items() if k == "oracle" or k.startswith("oracle.")}
    for k in saved:
        del sys.modules[k]
    sys.path.insert(0, pkg_parent)
    try:
        rng_t = _load(os.path.join(TESTS, "test_oracle_rng.py"), "_mut_rng_t")
        lupp_t = _load(os.path.join(TESTS, "test_oracle_lupp.py"), "_mut_lupp_t")
        icur_t = _load(os.path.join(TESTS, "test_oracle_icur.py"), "_mut_icur_t")
        rep_t = _load(os.path.join(TESTS, "test_oracle_replay.py"), "_mut_rep_t")
        qr_t = _load(os.path.join(TESTS, "test_oracle_qrcp.py"), "_mut_qr_t")
        srtt_t = _load(os.path.join(TESTS, "test_oracle_srtt.py"), "_mut_srtt_t")
        risk_t = _load(os.path.join(TESTS, "test_oracle_risk.py"), "_mut_risk_t")
        checks = [
            lambda: [rng_t.test_philox_known_answers(*k) for k in rng_t.PHILOX_KAT],
            rng_t.test_bf16_rounding_round_to_nearest_even,
            lambda: rng_t.test_sparse_sign_columns_have_distinct_rows(35, 8),
            lambda: [lupp_t.test_matches_brute_force_determinants(s) for s in range(8)],
            lambda: lupp_t.test_matches_lapack_getrf(0, (300, 55)),
            icur_t.test_sketch_rows,
            icur_t.test_example_3_1_worked_example,
            icur_t.test_dependent_selection_avoids_singular_core,
            lambda: icur_t.test_residuals_match_closed_forms_and_schur_zeros(0),
            lambda: icur_t.test_exact_recovery_of_exactly_low_rank(0),
            lambda: icur_t.test_estimator_within_factor_two_and_tolerance_met(0, "planted"),
            icur_t.test_sketch_products_follow_their_definitions,
            lambda: [rep_t.test_lupp_replay_values_are_determinant_ratios(s) for s in range(3)],
            lambda: rep_t.test_replaying_its_own_choices_reproduces_the_run("lupp", 0),
            lambda: rep_t.test_replaying_its_own_choices_reproduces_the_run("qrcp", 0),
            rep_t.test_qrcp_replay_values_are_volume_ratios,
            lambda: qr_t.test_matches_lapack_geqp3(1, (35, 500)),
            lambda: [qr_t.test_matches_brute_force_volumes(s) for s in range(3)],
            lambda: srtt_t.test_matches_fft_dct_of_signed_input(97, 11, 3),
            lambda: srtt_t.test_matches_fft_dct_of_signed_input(1000, 55, 0),
            srtt_t.test_rows_are_distinct_sorted_and_uniform,
            lambda: [srtt_t.test_full_transform_is_orthogonal(m) for m in (1, 7, 64)],
            lambda: [risk_t.test_denominator_a_is_the_rescaled_estimate(k) for k in (0, 1, 2)],
        ]
        for chk in checks:
            try:
                chk()
            except Exception:
                return False
        return True
    finally:
        sys.path.remove(pkg_parent)
        for k in [k for k in sys.modules if k == "oracle" or k.startswith("oracle.")]:
            del sys.modules[k]
        sys.modules.update(saved)


def _copy_oracle(tmp_path):
    dst = tmp_path / "oracle"
    shutil.copytree(os.path.join(ROOT, "oracle"), dst,
                    ignore=shutil.ignore_patterns("__pycache__", "*.so", "*.o"))
    return dst


def test_unmutated_copy_passes(tmp_path):
    _copy_oracle(tmp_path)
    assert _pins_pass(str(tmp_path))


@pytest.mark.parametrize("fname,old,new", MUTATIONS, ids=[f"{m[0]}:{i}" for i, m in enumerate(MUTATIONS)])
def test_planted_mistake_is_caught(tmp_path, fname, old, new):
    dst = _copy_oracle(tmp_path)
    path = dst / fname
    src = path.read_text()
    assert src.count(old) == 1, "mutation anchor not found: " + old
    path.write_text(src.replace(old, new))
    assert not _pins_pass(str(tmp_path))
