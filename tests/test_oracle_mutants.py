"""Planted mistakes in the CPU oracle must fail its pins (runs without a GPU).

Each case below copies the oracle's C source, makes one plausible slip in it
(a dropped term or factor, a wrong sign, an index off by one, a wrong
parity or normalisation, a transposed or missing mirror), builds the copy
with the oracle's own compiler flags and runs the pins of
tests/test_oracle.py against it in a fresh process.  The pins pass for an
unaltered copy built the same way (the control) and must fail for every
altered one.  The altered copies live in a temporary directory; the oracle
itself is never changed.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
ORACLE = os.path.join(ROOT, "oracle")
PINS = os.path.join(HERE, "test_oracle.py")

C, H = "dlt_oracle.c", "dlt_oracle_impl.h"

# (name, file, anchor, old, new): replace the first `old` after `anchor`
# (anchor None: `old` must occur exactly once in the file)
MUTANTS = [
    # nodes and weights (Sec. 2.1-2.2)
    ("nodes: Reinsch step sign", C, "static void leg_pair_ld",
     "d = ((LD)n * d - (LD)(2 * n + 1) * u * p)", "d = ((LD)n * d + (LD)(2 * n + 1) * u * p)"),
    ("nodes: Reinsch step index", C, "static void leg_pair_ld",
     "(LD)(2 * n + 1) * u * p) / (LD)(n + 1)", "(LD)(2 * n + 1) * u * p) / (LD)(n + 2)"),
    ("weights: dropped sin factor", C, None, "*w = 2 * st * st / (q * q);", "*w = 2 * st / (q * q);"),
    ("weights: derivative degree", C, None, "LD q = (LD)N * (cosl(t) * pN - pN1);",
     "LD q = (LD)(N + 1) * (cosl(t) * pN - pN1);"),
    ("nodes: missing mirror", C, None, "if (kk != k) t = PI_LD - t;", "if (kk != k) t = t;"),
    ("nodes: odd middle root", C, None, "t = PI_LD / 2; /*", "t = PI_LD / 2 + 1e-3L; /*"),
    # DLT, eq. (1)
    ("dlt: dropped c_0", H, "int FN(orc_dlt)", "REAL acc = (REAL)c[0];", "REAL acc = 0;"),
    ("dlt: coefficient index (u form)", H, "int FN(orc_dlt)",
     "acc += (REAL)c[n + 1] * (sg * p);", "acc += (REAL)c[n] * (sg * p);"),
    ("dlt: three-term recurrence (x form)", H, "int FN(orc_dlt)",
     "REAL pn = ((REAL)(2 * n + 1) * x * p - (REAL)n * pm)", "REAL pn = ((REAL)(2 * n + 1) * x * p + (REAL)n * pm)"),
    ("dlt: no parity sign past pi/2", H, "int FN(orc_dlt)", "if (flip) sg = -sg;", "if (flip) sg = sg;"),
    # NDCT, eqs. (3)-(4)
    ("ndct: first difference sign", H, "int FN(orc_ndct)", "REAL p = 1, d = -u;", "REAL p = 1, d = u;"),
    ("ndct: dropped factor 2 (u form)", H, "int FN(orc_ndct)", "d = d - 2 * u * p;", "d = d - u * p;"),
    ("ndct: Chebyshev recurrence sign (x form)", H, "int FN(orc_ndct)",
     "REAL pn = 2 * x * p - pm;", "REAL pn = 2 * x * p + pm;"),
    # IDLT, eq. (2)
    ("idlt: dropped weights", H, "int FN(orc_idlt)", "g[j] = (REAL)w[k] * (REAL)f[k];", "g[j] = (REAL)f[k];"),
    ("idlt: normalisation n + 1", H, "int FN(orc_idlt)",
     "c[i] = (double)(((REAL)n + (REAL)0.5) * tot[n]);", "c[i] = (double)(((REAL)n + (REAL)1.0) * tot[n]);"),
    ("idlt: dropped degree-0 term", H, "static void FN(idlt_group)", "a[0] += FN(idlt_gsum)(g);", "a[0] += 0;"),
    ("idlt: last node of each thread dropped", H, "int FN(orc_idlt)",
     "if (kg + j < k1) {", "if (kg + j + 1 < k1) {"),
    ("idlt: Reinsch step sign", H, "static void FN(idlt_group)",
     "q[j] = ((REAL)n * q[j] - (REAL)(2 * n + 1) * v[j] * p[j])",
     "q[j] = ((REAL)n * q[j] + (REAL)(2 * n + 1) * v[j] * p[j])"),
    ("idlt: textbook recurrence sign", H, "static void FN(idlt_group)",
     "REAL pn = ((REAL)(2 * n + 1) * v[j] * p[j] - (REAL)n * q[j])",
     "REAL pn = ((REAL)(2 * n + 1) * v[j] * p[j] + (REAL)n * q[j])"),
    ("idlt: pairwise group sum stops early", H, "static REAL FN(idlt_gsum)",
     "for (int h = IDLT_G / 2; h >= 1; h /= 2)", "for (int h = IDLT_G / 2; h >= 2; h /= 2)"),
    ("idlt: node of the other form counted too", H, "int FN(orc_idlt)",
     "gm[j] = (form[j] == fm) ? g[j] : 0;", "gm[j] = (form[j] >= 0) ? g[j] : 0;"),
    # Legendre values
    ("legendre: odd-degree mirror parity", H, "static void FN(leg_row)",
     "for (int64_t n = 1; n < N; n += 2) P[n] = -P[n];", "for (int64_t n = 0; n < N; n += 2) P[n] = -P[n];"),
    # leg2cheb, Sec. 3 eq. (9)
    ("Lambda: ratio", H, "static void FN(lam_table)",
     "v = v * ((long double)z + 0.5L)", "v = v * ((long double)z + 1.5L)"),
    ("Lambda: start value", H, "static void FN(lam_table)",
     "long double v = sqrtl(", "long double v = 2 * sqrtl("),
    ("leg2cheb: eps_0 = 2", H, "int FN(orc_leg2cheb)(", "REAL e = (k == 0) ? 1 : 2;", "REAL e = 2;"),
    ("leg2cheb: parity pattern", H, "int FN(orc_leg2cheb)(",
     "for (int64_t n = k; n < N; n += 2)", "for (int64_t n = k; n < N; n += 1)"),
    ("leg2cheb: transposed Lambda argument", H, "int FN(orc_leg2cheb)(",
     "(L[(n - k) / 2] * L[(n + k) / 2])", "(L[(n - k) / 2] * L[(n - k) / 2])"),
    ("leg2cheb rows: dropped diagonal", H, "int FN(orc_leg2cheb_rows)",
     "for (int64_t n = k; n < N; n += 2)", "for (int64_t n = k + 2; n < N; n += 2)"),
    ("cheb2leg: diagonal entry", H, "int FN(orc_cheb2leg)",
     "REAL diag = e / PI_R * (REAL)(L[0] * L[k]);", "REAL diag = e / PI_R * (REAL)(L[0] * L[0]);"),
    ("cheb2leg: off-diagonal start", H, "int FN(orc_cheb2leg)",
     "for (int64_t n = k + 2; n < N; n += 2)", "for (int64_t n = k + 4; n < N; n += 2)"),
    ("leg2cheb_t: dropped diagonal", H, "int FN(orc_leg2cheb_t)",
     "for (int64_t k = n & 1; k <= n; k += 2)", "for (int64_t k = n & 1; k < n; k += 2)"),
    ("leg2cheb_t: eps on the wrong index", H, "int FN(orc_leg2cheb_t)",
     "REAL e = (k == 0) ? 1 : 2;", "REAL e = (n == 0) ? 1 : 2;"),
]


def _mutate(text, anchor, old, new):
    if anchor is None:
        assert text.count(old) == 1, old
        return text.replace(old, new)
    assert text.count(anchor) == 1, anchor
    a = text.index(anchor)
    i = text.index(old, a)
    return text[:i] + new + text[i + len(old):]


# runs the pins with the oracle package pointed at another build of it
_DRIVER = (
    "import sys; sys.path.insert(0, sys.argv[1]); import oracle; oracle._build.LIB = sys.argv[2]; "
    "import pytest; sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', sys.argv[3]]))"
)


def _build_and_pin(tmp, tag, edit):
    sys.path.insert(0, ROOT)
    from oracle import build as ob

    d = os.path.join(tmp, tag)
    os.makedirs(d)
    for f in (C, H):
        shutil.copy(os.path.join(ORACLE, f), d)
    if edit is not None:
        fname, anchor, old, new = edit
        p = os.path.join(d, fname)
        with open(p) as fh:
            text = fh.read()
        with open(p, "w") as fh:
            fh.write(_mutate(text, anchor, old, new))
    lib = os.path.join(d, "liboracle.so")
    ob.compile_lib(os.path.join(d, C), lib)
    env = dict(os.environ, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-c", _DRIVER, ROOT, lib, PINS], capture_output=True, text=True,
                       env=env, timeout=300)
    return r.returncode, (r.stdout + r.stderr)[-600:]


@pytest.mark.slow
def test_planted_mistakes_fail_the_pins(tmp_path):
    tmp = str(tmp_path)
    jobs = {"control": None}
    for i, (name, f, anchor, old, new) in enumerate(MUTANTS):
        jobs[f"m{i:02d} {name}"] = (f, anchor, old, new)
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        futs = {k: ex.submit(_build_and_pin, tmp, f"case{i}", e) for i, (k, e) in enumerate(jobs.items())}
        res = {k: f.result() for k, f in futs.items()}
    rc, out = res.pop("control")
    assert rc == 0, "the unaltered copy must pass the pins:\n" + out
    survived = [k for k, (rc, _) in res.items() if rc != 1]
    assert not survived, "planted mistakes not caught by any pin (or not built): " + ", ".join(
        f"{k} (exit {res[k][0]}): {res[k][1][-200:]}" for k in survived)
