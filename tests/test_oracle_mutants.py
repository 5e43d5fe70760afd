"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a copy of the C oracle (on the CPU), builds
it, and runs the oracle pin suite (tests/test_oracle.py) against the mutant in
a subprocess: the suite has to fail.  Section references are to arXiv
2604.06602.
"""
from __future__ import annotations

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "umi_oracle.c")

MUTANTS = {
    "alpha dropped (Eq. 2)": ("double u_eff = (u < 0.0) ? alpha * u : u;", "double u_eff = u;"),
    "alpha on the upper side (Eq. 2)": ("double u_eff = (u < 0.0) ? alpha * u : u;",
                                        "double u_eff = (u > 0.0) ? alpha * u : u;"),
    "weight not squared (Eq. 3)": ("        return t * t;\n    }\n    return 0.0;", "        return t;\n    }\n    return 0.0;"),
    "scale constant inverted (Section 2.2)": ("#define ORACLE_SCALE_CONST 0.6745", "#define ORACLE_SCALE_CONST 1.4826"),
    "upper set not strict (Eq. 1)": ("if (xi > m) { /* strictly above", "if (xi >= m) { /* strictly above"),
    "upper RMS over n, not n+ (Eq. 1)": ("sqrt(sum_sq / (double)n_plus)", "sqrt(sum_sq / (double)n)"),
    "upper median instead of lower": ("keys[(n - 1) / 2]", "keys[n / 2]"),
    "negative values ordered wrongly": ("return (b & 0x80000000u) ? ~b : (b | 0x80000000u);",
                                        "return (b & 0x80000000u) ? b : (b | 0x80000000u);"),
    "c dropped from u (Section 2.3)": ("double cs = c * s;", "double cs = s;"),
    "unweighted sum in Eq. 4": ("swx += w * xi;", "swx += xi;"),
    "one iteration too many": ("for (int it = 0; it < iters; ++it)", "for (int it = 0; it <= iters; ++it)"),
    "window one sample too wide": ("int64_t h = (W - 1) / 2;", "int64_t h = (W + 1) / 2;"),
    "gap measured from segment start": ("(time[q] - time[last]) > ORACLE_GAP_DAYS", "(time[q] - time[lo]) > ORACLE_GAP_DAYS"),
    "minimum segment W/2 instead of W/3": ("int64_t m_min = W / 3;", "int64_t m_min = W / 2;"),
    "invalid samples kept in windows": ("        if (!sample_valid(flux, time, q)) continue;\n        /* reading R19", "        if (0) continue;\n        /* reading R19"),
    "MAD: upper median of deviations": ("double s = dev[(n - 1) / 2];", "double s = dev[n / 2];"),
    "MAD: scaled to sigma": ("double s = dev[(n - 1) / 2];", "double s = 1.4826 * dev[(n - 1) / 2];"),
    "MAD: deviations not absolute": ("dev[i] = fabs((double)x[i] - m);", "dev[i] = (double)x[i] - m;"),
    "per-curve alpha ignored": ("job->W[b], job->alpha[b], job->c[b],", "job->W[b], job->alpha[0], job->c[b],"),
    "normalise inverted": ("(double)flux[j] / trend[j];", "trend[j] / (double)flux[j];"),
    "time window uses the full length as half-width": ("fabs(time[q] - time[i]) <= 0.5 * window_days", "fabs(time[q] - time[i]) <= window_days"),
    "time window ignored": ("if (window_days > 0.0 && !(fabs", "if (window_days > 1e300 && !(fabs"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not found uniquely: %r" % old
    mut = tmp_path / "umi_oracle_mutant.c"
    mut.write_text(src.replace(old, new))
    sys.path.insert(0, ROOT)
    from oracle.oracle import compile_oracle
    lib = compile_oracle(str(mut), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, UMI_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "pins did not catch: %s\n%s" % (name, r.stdout[-2000:])


# Mistakes in the estimate of one window that the hand-worked trajectories
# and the white-noise bias pin must catch on their own (without the rest of
# the suite): every iterate of a worked window moves under each of them.
WINDOW_MUTANTS = [
    "alpha dropped (Eq. 2)", "alpha on the upper side (Eq. 2)", "weight not squared (Eq. 3)",
    "scale constant inverted (Section 2.2)", "upper set not strict (Eq. 1)",
    "upper RMS over n, not n+ (Eq. 1)", "upper median instead of lower",
    "negative values ordered wrongly", "c dropped from u (Section 2.3)",
    "unweighted sum in Eq. 4", "one iteration too many",
]


@pytest.mark.parametrize("name", WINDOW_MUTANTS)
def test_trajectory_pins_alone_catch_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    mut = tmp_path / "umi_oracle_mutant.c"
    mut.write_text(src.replace(old, new))
    sys.path.insert(0, ROOT)
    from oracle.oracle import compile_oracle
    lib = compile_oracle(str(mut), str(tmp_path / "libmutant.so"))
    env = dict(os.environ, UMI_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        "-k", "hand_worked_trajectories or white_noise_bias_matches",
                        os.path.join(ROOT, "tests", "test_oracle.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and " failed" in r.stdout, \
        "trajectory pins did not catch: %s\n%s" % (name, r.stdout[-2000:])
