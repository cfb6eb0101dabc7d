"""Each plausible mistake planted in the oracle must fail at least one pin.

The oracle source is copied to a temporary directory, one edit is applied, the
copy is compiled, and the pin battery of tests/_pins.py is run against it.  This
shows that the pins constrain every part of the rotation, the sweep, the final
eigenvalues and their order.  Nothing here touches the GPU."""
import os
import shutil

import numpy as np
import pytest

import oracle
from _pins import battery

MUTATIONS = {
    # the sign of sigma as printed (same-sign pairs become hyperbolic)
    "printed_hyp_sign": ("RT sigma = (RT)(jr * js);", "RT sigma = (RT)(-jr * js);"),
    "theta_inner_sign": ("(ass - sigma * arr)", "(ass + sigma * arr)"),
    "theta_swapped_diag": ("(ass - sigma * arr)", "(arr - sigma * ass)"),
    "update_sign": ("gr[k] = cs * f - sigma * sn * g;", "gr[k] = cs * f + sigma * sn * g;"),
    # the second assignment as printed targets g_r
    "printed_second_target": ("gs[k] = sn * f + cs * g;", "gr[k] = sn * f + cs * g;"),
    "phase_conjugated": ("ST f = phase * gr[k];", "ST f = CONJ(phase) * gr[k];"),
    "transposed_dot": ("s += CONJ(x[k]) * y[k];", "s += x[k] * CONJ(y[k]);"),
    "dropped_eta_sign": ("RT eta = FN(sgn)(re_ars) * abs_ars;", "RT eta = abs_ars;"),
    "hyperbolic_cosine_as_trig": ("cs = 1 / R_SQRT((1 - R_FABS(t)) * (1 + R_FABS(t)));",
                                  "cs = 1 / R_SQRT(1 + t * t);"),
    "larger_root": ("t = FN(sgn)(theta) / (at + R_SQRT(theta * theta + sigma));",
                    "t = FN(sgn)(theta) * (at + R_SQRT(theta * theta + sigma));"),
    "eigenvalue_sign_dropped": ("lam[i] = (RT)J[i] * d;", "lam[i] = d;"),
    "skips_adjacent_pairs": ("for (int s = r + 1; s < n; s++)", "for (int s = r + 2; s < n; s++)"),
    "ascending_sort": ("lam[idx[b]] < lam[key]", "lam[idx[b]] > lam[key]"),
    "eigenvector_wrong_column": ("ST v = nrm > 0 ? G[(size_t)c * m + i] / nrm : (ST)0;",
                                 "ST v = nrm > 0 ? G[(size_t)k * m + i] / nrm : (ST)0;"),
    "norm_missing_imag": ("s += CREAL(x[k]) * CREAL(x[k]) + CIMAG(x[k]) * CIMAG(x[k]);",
                          "s += CREAL(x[k]) * CREAL(x[k]);"),
}


def _solver(lib):
    def solve(G, J):
        return oracle.solve(G, J, lib=lib, max_sweeps=40)
    return solve


def test_unmutated_oracle_passes_battery():
    assert battery(_solver(oracle.load())) == []


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_mutation_is_caught(name, tmp_path):
    old, new = MUTATIONS[name]
    src = os.path.dirname(oracle.__file__)
    for f in ("jj_oracle.c", "jj_oracle_body.inc", "jj_bp_body.inc"):
        shutil.copy(os.path.join(src, f), tmp_path / f)
    body = (tmp_path / "jj_oracle_body.inc").read_text()
    assert body.count(old) >= 1, "mutation target not found in the oracle source"
    (tmp_path / "jj_oracle_body.inc").write_text(body.replace(old, new))
    so = str(tmp_path / "libmut.so")
    oracle.build(out=so, src_dir=str(tmp_path))
    lib = oracle.load(so)
    with np.errstate(all="ignore"):
        fails = battery(_solver(lib))
    assert fails, "planted mistake %r was not caught by any pin" % name
