"""The oracle's pins must catch plausible mistakes in the oracle itself.

Each case plants one mistake in a private copy of one of the oracle's C sources (a flipped sign, a wrong
or transposed operand, a dropped term or factor, a changed comparison or filter tap), rebuilds
that copy with gcc and runs the oracle pin tests against it: at least one pin must fail.  The
working tree is never touched; every copy lives in a temporary directory."""
import concurrent.futures as cf
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["tests/test_oracle_degraf.py", "tests/test_oracle_pyramid.py", "tests/test_oracle_rlof.py",
             "tests/test_oracle_illum.py", "tests/test_oracle_grad.py", "tests/test_oracle_detect_grad.py",
             "tests/test_oracle_next3.py"]

# (name, original text, planted text): the first occurrence in degraf_oracle.c is replaced
MUTATIONS = [
    ("selection tie goes to the negative centroid (Eq. 2 rule)",
     "int neg = s_neg > s_pos;", "int neg = s_neg >= s_pos;"),
    ("row moment takes the column index (Eq. 1)",
     "i_pos += (int64_t)i * v;", "i_pos += (int64_t)j * v;"),
    ("pyramid taps 1 5 4 5 1 (same sum)",
     "static const int k5[5] = {1, 4, 6, 4, 1};", "static const int k5[5] = {1, 5, 4, 5, 1};"),
    ("bilinear interpolation with the two off-diagonal taps swapped",
     "double h0 = i00 + fx * (i10 - i00), h1 = i01 + fx * (i11 - i01);",
     "double h0 = i00 + fx * (i01 - i00), h1 = i10 + fx * (i11 - i10);"),
    ("psi without its sigma1 factor in the middle band",
     "return copysign(s1 * (s2 - a) / (s2 - s1), r);", "return copysign((s2 - a) / (s2 - s1), r);"),
    ("off-diagonal of the structure tensor with the wrong sign",
     "b += gxk[k] * gyk[k];", "b -= gxk[k] * gyk[k];"),
    ("vertical template gradient taken along x",
     "gyk[k] = 0.5 * (or_bilinear(I0l, Wl, Hl, x, y + 1.0) - or_bilinear(I0l, Wl, Hl, x, y - 1.0));",
     "gyk[k] = 0.5 * (or_bilinear(I0l, Wl, Hl, x + 1.0, y) - or_bilinear(I0l, Wl, Hl, x - 1.0, y));"),
    ("2x2 solve with the right-hand side transposed",
     "double stepX = (C * bx - B * by) / det;", "double stepX = (C * by - B * bx) / det;"),
    ("no least-squares fallback when the weighted system is near singular",
     "if (!(det > 1e-6 * det0)) {", "if (0) {"),
    ("guess not doubled from one level to the next",
     "gX = 2.0 * (gX + dX);", "gX = (gX + dX);"),
    ("illumination offset entering the residual with the wrong sign",
     "double res = J - (1.0 + m) * T[k] - c;", "double res = J - (1.0 + m) * T[k] + c;"),
    ("adjoint without the template-gradient term of dI0",
     "dI0[ixp[t]] += cx * wxp[t];", "(void)cx;"),
    ("cross arms that stop at a difference equal to the threshold",
     "while (left < re && fabs(row[re - left - 1] - a) <= tau) ++left;",
     "while (left < re && fabs(row[re - left - 1] - a) < tau) ++left;"),
    ("illumination model on supports of fewer than four pixels",
     "if (!(lam_min / (double)nsup >= o->min_eig) || nsup < 4) {", "if (!(lam_min / (double)nsup >= o->min_eig)) {"),
    ("illumination model carrying a runaway gain to the next level",
     "if (!bad && l > lstop && !(1.0 + m >= 0.25 && 1.0 + m <= 4.0)) bad = 1;", "(void)0;"),
    ("cross region decided one pixel to the right of the point's cell",
     "I[(int64_t)clampi(y0 + ky, 0, H - 1) * W + clampi(x0 + kx, 0, W - 1)];",
     "I[(int64_t)clampi(y0 + ky, 0, H - 1) * W + clampi(x0 + kx + 1, 0, W - 1)];"),
    ("cross support without the erosion by the gradient stencil",
     "const uint8_t in = R[q] & R[q - 1] & R[q + 1] & R[q - e] & R[q + e];", "const uint8_t in = R[q];"),
    ("trackability divided by the window instead of the support",
     "if (!(lam_min / (double)nsup >= o->min_eig)) {", "if (!(lam_min / (double)npix >= o->min_eig)) {"),
    ("gradient of the robust equation at a point the tracker stopped on its least-squares step",
     "const double s1 = ls ? INFINITY : sigma1, s2 = ls ? INFINITY : sigma2;\n\n        /* J = sum psi' g (grad J)^T */",
     "const double s1 = sigma1, s2 = sigma2;\n        (void)ls;\n\n        /* J = sum psi' g (grad J)^T */"),
    ("illumination-model gradient of the robust equations in the least-squares regime",
     "const int ls = ls_regime_illum(I0, I1, W, H, px, py, r, ux, uy, m, c, sigma1, sigma2);",
     "const int ls = 0;"),
    ("global fit weights without the square of the Tukey factor",
     "w[i] = (e < c) ? (1.0 - t * t) * (1.0 - t * t) : 0.0;", "w[i] = (e < c) ? (1.0 - t * t) : 0.0;"),
    ("global prior start not scaled to the coarsest level",
     "init[2 * i] = (A[0] * x + A[1] * y + A[2]) / top;", "init[2 * i] = (A[0] * x + A[1] * y + A[2]);"),
]

# the same for the dense interpolation's oracle, checked by its own pins
EPIC_PIN_FILES = ["tests/test_oracle_epic.py"]
EPIC_MUTATIONS = [
    ("edge map without its vertical term",
     "E[(int64_t)y * W + x] = abs(gx) + abs(gy);", "E[(int64_t)y * W + x] = abs(gx);"),
    ("geodesic step cost without the edge value of the pixel entered",
     "const int64_t c = it.k0 + kappa + E[p] + E[q];", "const int64_t c = it.k0 + kappa + E[p];"),
    ("equal distances go to the higher seed index",
     "(c == D[q] && it.k1 < L[q])", "(c == D[q] && it.k1 > L[q])"),
    ("seed-graph edge length without the far side's distance",
     "const int64_t w = D[p] + kappa + E[p] + E[q] + D[q];", "const int64_t w = D[p] + kappa + E[p] + E[q];"),
    ("affine fit rows scaled by the weight instead of its square root",
     "const double r = sqrt(exp2(-(double)nd[j] / (double)h));", "const double r = exp2(-(double)nd[j] / (double)h);"),
]


def _copy_tree(dst):
    ign = shutil.ignore_patterns("__pycache__", "*.so", "*.o", "_build", "*.tmp", "csrc")
    for d in ("oracle", "tests", "paper_1901_09971_amd"):
        shutil.copytree(os.path.join(ROOT, d), os.path.join(dst, d), ignore=ign)


def _run_mutant(tmp, old, new, source="degraf_oracle.c", pins=PIN_FILES):
    src_path = os.path.join(tmp, "oracle", source)
    if old is not None:
        src = open(src_path).read()
        assert src.count(old) >= 1, f"mutation target not found: {old}"
        open(src_path, "w").write(src.replace(old, new, 1))
    env = dict(os.environ, OMP_NUM_THREADS="2", PYTHONDONTWRITEBYTECODE="1")
    p = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pins],
                       cwd=tmp, env=env, capture_output=True, text=True, timeout=900)
    return p.returncode, (p.stdout + p.stderr).strip().splitlines()


def test_every_planted_mistake_fails_a_pin(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    cases = [(m, "degraf_oracle.c", PIN_FILES) for m in MUTATIONS]
    cases += [(m, "epic_oracle.c", EPIC_PIN_FILES) for m in EPIC_MUTATIONS]
    dirs = []
    for i in range(len(cases) + 1):
        d = str(tmp_path / f"m{i}")
        _copy_tree(d)
        dirs.append(d)
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        # the unchanged copy is the control: all its pins must pass
        control = ex.submit(_run_mutant, dirs[-1], None, None, "degraf_oracle.c", PIN_FILES + EPIC_PIN_FILES)
        futs = [ex.submit(_run_mutant, d, old, new, src, pins)
                for d, ((_, old, new), src, pins) in zip(dirs, cases)]
        results = [f.result() for f in futs]
        rc0, lines0 = control.result()
    assert rc0 == 0, lines0[-5:]
    survivors = []
    for ((name, _, _), _, _), (rc, lines) in zip(cases, results):
        last = lines[-1] if lines else ""
        print(f"{name}: rc={rc} {last}", flush=True)
        # a pin must fail (not a build or collection error)
        if not (rc == 1 and " failed" in last and "error" not in last):
            survivors.append((name, rc, last))
    assert not survivors, survivors
