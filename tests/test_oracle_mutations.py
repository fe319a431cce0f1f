"""Planted mistakes in the oracle must be caught by its pins.

Each case copies oracle.c, applies one plausible mistake (a sign, a dropped
term, a swapped index, a wrong convention), builds it on the CPU and runs the
pin suite against it; the suite must fail.  This shows the pins constrain
every part of the oracle, not just that the current build passes them.
"""
import os
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTATIONS = [
    ("type1 sign of the x phase", "ex[2 * i + 1] = -sin(k * x[j]);", "ex[2 * i + 1] = sin(k * x[j]);"),
    ("type1 complex product", "row[2 * i + 1] += yr * xi + yi * xr;", "row[2 * i + 1] += yr * xi - yi * xr;"),
    ("mode box offset", "static int mode_lo(int N) { return -(N / 2); }", "static int mode_lo(int N) { return -((N - 1) / 2); }"),
    ("window dropped from the strength", "return w * W * h;", "return w * h;"),
    ("Hann sign", "*W = 0.5 * (1.0 + cos(u));", "*W = 0.5 * (1.0 - cos(u));"),
    ("Hann gradient transposed", "*dWdy = g * dy;", "*dWdy = g * dx;"),
    ("product-set sum sign of the y phase", "ey[2 * r + 1] = -c[j] * sin(ph);",
     "ey[2 * r + 1] = c[j] * sin(ph);"),
    ("reconstruction phase sign", "s += cc[2 * m] * cos(ph) - cc[2 * m + 1] * sin(ph);",
     "s += cc[2 * m] * cos(ph) + cc[2 * m + 1] * sin(ph);"),
    ("reconstruction target without the window", "const double t = W * h[j];", "const double t = h[j];"),
    ("spectral variance keeps the DC mode", "if (mode_lo(N1) + i == 0 && mode_lo(N2) + r == 0) continue;", ""),
    ("physical variance without the weights", "kadd(&wt2, w[j] * t * t);", "kadd(&wt2, t * t);"),
    ("launch weight: intrinsic frequency from one wind component", "const double omega = -(k1 * ux + k2 * uy);",
     "const double omega = -(k1 * ux);"),
    ("launch weight: propagating band not enforced", "if (!(aw > fabs(fc) && aw < N)) return 0.0;", ""),
    ("launch weight: dispersion relation inverted",
     "const double m2 = kk * (N * N - omega * omega) / (omega * omega - fc * fc);",
     "const double m2 = kk * (omega * omega - fc * fc) / (N * N - omega * omega);"),
    ("flow records indexed by cell only", "const double *fl = flow + 6 * v;", "const double *fl = flow + 6 * c;"),
    ("scale dropped", "for (int64_t m = 0; m < 2 * M; ++m) out[m] *= scale;", ""),
    ("EMS tie-break reversed", "return (a->id < b->id) ? -1 : (a->id > b->id);", "return (a->id > b->id) ? -1 : (a->id < b->id);"),
    ("EMS participation ratio", "tot * tot / tot2", "tot / tot2"),
    ("EMS gap ratio inverted", "term = exp(-(a / b - 1.0) / delta);", "term = exp(-(b / a - 1.0) / delta);"),
    ("EMS S_delta normaliser", "sdel = acc / (double)(Jmax - 1);", "sdel = acc / (double)(Jmax);"),
    ("EMS N_eff clip dropped", "w1 * nclip / (double)Jmax", "w1 * neff / (double)Jmax"),
    ("EMS threshold off by one", "if (run / tot >= alphaC) { kc = j + 1; break; }", "if (run / tot >= alphaC) { kc = j + 2; break; }"),
    ("EMS no pairing", "if (use_pairs && !(kx == 0 && ky == 0)) {", "if (0) {"),
    ("EMS weight only on the representative",
     "const double op = mode_weight ? mode_weight[partner] : 1.0;", "const double op = 1.0;"),
    ("EMS weight squared",
     "e += om * (f[2 * idx] * f[2 * idx] + f[2 * idx + 1] * f[2 * idx + 1]);",
     "e += om * om * (f[2 * idx] * f[2 * idx] + f[2 * idx + 1] * f[2 * idx + 1]);"),
    ("EMS weight dropped",
     "const double om = mode_weight ? mode_weight[idx] : 1.0;", "const double om = 1.0;"),
    ("EMS k_min ignored", "int k = (kc > k_min) ? kc : k_min;", "int k = kc;"),
    ("adjoint x derivative sign", "sx += -kxv * im;", "sx += kxv * im;"),
    ("adjoint phase sign", "ey[2 * i + 1] = sin(k * y[j]);", "ey[2 * i + 1] = -sin(k * y[j]);"),
    ("adjoint grad_x uses y derivative", "(dWx * u + W * ux)", "(dWx * u + W * uy)"),
    ("adjoint window derivative dropped", "(dWy * u + W * uy)", "(W * uy)"),
    ("frame: shortest edge instead of the longest", "if (L > best) { best = L; m = i; }",
     "if (best < 0 || L < best) { best = L; m = i; }"),
    ("frame: rotation transposed", "ut[2 * i + 1] = -sn * dx + cs * dy;", "ut[2 * i + 1] = sn * dx + cs * dy;"),
    ("frame: half-width without the factor 1/2", "const double H = 0.5 * eta * fmax(ex, ey);",
     "const double H = eta * fmax(ex, ey);"),
    ("box coordinates without pi", "xb[j] = ux * M_PI / H;", "xb[j] = ux / H;"),
    ("circle area taken as the square's", "else if (mask == 2) area = M_PI * H * H;",
     "else if (mask == 2) area = 4.0 * H * H;"),
    ("triangle mask: edge test sign", "int neg = (d1 < 0) || (d2 < 0) || (d3 < 0);",
     "int neg = (d1 < 0) || (d2 > 0) || (d3 < 0);"),
    ("clipping: intersection parameter", "const double t = da / (da - db);", "const double t = db / (da - db);"),
    ("Voronoi: raster points outside the mask counted", "if (!in_mask(mask, gx, gy, H, ut)) continue;", ""),
    ("Voronoi: empty-cell floor dropped", "(double)n[j - a] : floor_frac)", "(double)n[j - a] : 0.0)"),
    ("deplaning by the unweighted mean of all samples", "hbar += wb[j] * h[j];", "hbar += h[j] / (double)(b - a);"),
]


@pytest.mark.parametrize("name,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_mutation(name, old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation site not unique: " + old
    with tempfile.TemporaryDirectory() as td:
        mut = os.path.join(td, "oracle_mut.c")
        lib = os.path.join(td, "liboracle_mut.so")
        open(mut, "w").write(src.replace(old, new))
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", lib, mut, "-lm"])
        env = dict(os.environ, ENUFFT_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
        r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                            os.path.join(ROOT, "tests", "test_oracle.py")],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode != 0, "pins did not catch: " + name
