"""The oracle's pins must catch plausible mistakes.

Each case plants one mistake in a private copy of the oracle source (on the
CPU, never on a GPU), builds it, and runs the pin suite against that build in a
subprocess; the suite must fail.  A mistake the pins did not catch would make
them too weak to trust the oracle.
"""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lpa_oracle.c")

# (name, original text, planted mistake)
MUTATIONS = [
    ("window not truncated", "const double k = (exp(-d2 / h) - k_edge) * kt;", "const double k = exp(-d2 / h) * kt;"),
    ("window exp(-d2/h^2)", "const double k = (exp(-d2 / h) - k_edge) * kt;",
     "const double k = (exp(-d2 / (h * h)) - exp(-r * r / (h * h))) * kt;"),
    ("weight 1/sigma", "orc_sample smp = {dx, dy, f, 1.0 / var, k};", "orc_sample smp = {dx, dy, f, 1.0 / sqrt(var), k};"),
    ("B without K^2", "const double w2 = s->k * s->k * s->ivar;", "const double w2 = s->k * s->ivar;"),
    ("basis dx*dy -> dx*dx", "phi[4] = dx * dy;", "phi[4] = dx * dx;"),
    ("offset sign", "const double dx = Xk - X, dy = Yk - Y;", "const double dx = X - Xk, dy = Yk - Y;"),
    ("affine transposed", "*X = a[0] * x + a[1] * y + a[2];", "*X = a[0] * x + a[3] * y + a[2];"),
    ("radiance without exposure", "const double f = (y - b) / (g * e * a);", "const double f = (y - b) / (g * a);"),
    ("variance gain not squared", "*var_hat = (g * g * e * a * shot + rv) / (g * g * e * e * a * a);",
     "*var_hat = (g * e * a * shot + rv) / (g * g * e * e * a * a);"),
    ("variance without readout", "*var_hat = (g * g * e * a * shot + rv) / (g * g * e * e * a * a);",
     "*var_hat = (g * g * e * a * shot + 1e-30) / (g * g * e * e * a * a);"),
    ("saturation exclusive", "if (y >= sat) return 0;", "if (y > sat) return 0;"),
    ("ICI strict tie", "if (lo_run <= hi_run)", "if (lo_run < hi_run)"),
    ("no equilibration", "At[i][j] = scale[i] * A[i][j] * scale[j];", "At[i][j] = A[i][j];"),
    ("back substitution index", "for (int k = i + 1; k < n; ++k) t -= L[k][i] * x[k];",
     "for (int k = i + 1; k < n; ++k) t -= L[i][k] * x[k];"),
    ("box too small", "const double wx = reff * sqrt(i00 * i00 + i01 * i01), wy = reff * sqrt(i10 * i10 + i11 * i11);",
     "const double wx = 0.5 * reff * sqrt(i00 * i00 + i01 * i01), wy = 0.5 * reff * sqrt(i10 * i10 + i11 * i11);"),
    ("default h", "2.0 * P->radii[m] * P->radii[m] / 9.0", "2.0 * P->radii[m] * P->radii[m] / 4.5"),
    ("green ratio not applied to radius", "const double r = P->radii[m] * kappa;", "const double r = P->radii[m];"),
    ("CFA GRBG wrong", "{1, 0, 2, 1}, /* GRBG */", "{1, 2, 0, 1}, /* GRBG */"),
    ("variance sandwich uses A", "var += g[i] * B[i][j] * g[j];", "var += g[i] * A[i][j] * g[j];"),
    ("fallback skipped", "for (int o = M; o >= 0; --o) {", "for (int o = M; o >= M; --o) {"),
    # adaptive anisotropic LPA / CALPA (Sec. 5.4, 5.5)
    ("steered window uses C inverse",
     "const double d2 = C ? C[0] * dx * dx + 2.0 * C[1] * dx * dy + C[2] * dy * dy : dx * dx + dy * dy;",
     "const double d2 = C ? (C[2] * dx * dx - 2.0 * C[1] * dx * dy + C[0] * dy * dy) / (C[0] * C[2] - C[1] * C[1])"
     " : dx * dx + dy * dy;"),
    ("window elongated across the edge", "double la = gamma * sigma, lb = gamma / sigma;",
     "double la = gamma / sigma, lb = gamma * sigma;"),
    ("steering from the edge direction", "const double u1x = cos(phi), u1y = sin(phi);",
     "const double u1x = -sin(phi), u1y = cos(phi);"),
    ("elongation without lambda1", "const double sigma = (s1 + A->lambda1) / (s2 + A->lambda1);",
     "const double sigma = (s1 + 1e-300) / (s2 + 1e-300);"),
    ("scaling without the sample count", "pow((s1 * s2 + A->lambda2) / (double)count, A->alpha)",
     "pow(s1 * s2 + A->lambda2, A->alpha)"),
    ("analysis window short by a row", "for (int b = -q; b <= q; ++b) {", "for (int b = -q + 1; b <= q; ++b) {"),
    ("steering eigenvalue not clamped", "la = la < lo ? lo : (la > hi ? hi : la);", "la = la * 1.0;"),
    ("gradients of the R channel",
     "gather_support(sensors, n_sensors, raw, X, Y, 1, r, h, NULL, P->exhaustive, 1, 0.0, &list)",
     "gather_support(sensors, n_sensors, raw, X, Y, 0, r, h, NULL, P->exhaustive, 1, 0.0, &list)"),
    ("ellipse box not widened", "reff = r / sqrt(lmin);", "reff = r;"),
    # per-pixel calibration frames (Sec. 6)
    ("non-uniformity not in the radiance", "const double f = (y - b) / (g * e * a);",
     "const double f = (y - b) / (g * e);"),
    ("non-uniformity power in the variance", "(g * g * e * e * a * a)", "(g * g * e * e * a)"),
    ("bias frame ignored", "const double b = pix && s->bias ? s->bias[i] : s->black_level;",
     "const double b = s->black_level;"),
    ("readout variance frame ignored",
     "const double rv = pix && s->read_var ? s->read_var[i] : s->read_sigma * s->read_sigma;",
     "const double rv = s->read_sigma * s->read_sigma;"),
    ("saturation frame ignored", "const double sat = pix && s->sat ? s->sat[i] : s->saturation;",
     "const double sat = s->saturation;"),
    # temporal LPA (T1-T4)
    ("temporal weight one frame late", "exp(-(double)t * t / h_t)", "exp(-(double)(t + 1) * (t + 1) / h_t)"),
    ("temporal weight outside the truncation", "const double k = (exp(-d2 / h) - k_edge) * kt;",
     "const double k = exp(-d2 / h) * kt - k_edge;"),
    ("frames indexed sensor-major", "raw + (size_t)t * n_sensors, X, Y", "raw + (size_t)t, X, Y"),
    ("zero temporal scale keeps every frame", "(h_t > 0.0 ? exp(-(double)t * t / h_t) : 0.0)",
     "(h_t > 0.0 ? exp(-(double)t * t / h_t) : 1.0)"),
    # rounding-sensitivity diagnostics
    ("sens_y without the b terms", "    sy += fabs(g[i]) * ba[i];\n", "\n"),
    ("sens_y without the A terms", "sy += fabs(g[i]) * Aa[i][j] * fabs(C[j]);", "sy += 0.0 * Aa[i][j];"),
    ("sens_v without the factor 2", "sv += 2.0 * fabs(Bg[i])", "sv += fabs(Bg[i])"),
    ("sens_v with signed A", "q += Aa[i][j] * fabs(g[j]);", "q += A[i][j] * g[j];"),
    ("l1f without the window", "l1f += fabs(gp * s->k * s->ivar * s->f);", "l1f += fabs(gp * s->ivar * s->f);"),
    ("defect mask ignored", "if (pix && s->defect && s->defect[i]) return 0;", "if (0) return 0;"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,bad", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(name, orig, bad):
    with open(SRC) as fh:
        text = fh.read()
    assert text.count(orig) >= 1, f"mutation anchor not found: {orig}"
    mutated = text.replace(orig, bad, 1)
    with tempfile.TemporaryDirectory() as tmp:
        src = os.path.join(tmp, "lpa_oracle.c")
        with open(src, "w") as fh:
            fh.write(mutated)
        shutil.copy(os.path.join(ROOT, "oracle", "lpa_oracle.h"), tmp)
        lib = os.path.join(tmp, "libmut.so")
        subprocess.run(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-ffp-contract=off", "-o", lib,
                        src, "-lm"], check=True)
        env = dict(os.environ, LPA_ORACLE_LIB_OVERRIDE=lib)
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                            os.path.join(ROOT, "tests", "test_oracle_calpa.py"),
                            os.path.join(ROOT, "tests", "test_oracle_calib.py"),
                            os.path.join(ROOT, "tests", "test_oracle_temporal.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"planted mistake '{name}' passed every pin:\n{r.stdout[-2000:]}"
