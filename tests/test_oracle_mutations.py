"""Planted mistakes: each mutant of the oracle (a dropped term, a wrong sign,
a wrong index, a transposed operand, a wrong constant) must fail the pin
suite.  Built and run on the CPU only."""
import os
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "spx_oracle.c")

MUTANTS = {
    "skew sign": ("y[i] = x[i] + t;", "y[i] = x[i] - t;"),
    "skew factor": ("return (sqrt((double)n + 1.0) - 1.0) / (double)n;",
                    "return (sqrt((double)n + 1.0) - 1.0) / (double)(n + 1);"),
    "scale direction": ("/ orc_adjust_scale(n));", "* orc_adjust_scale(n));"),
    "sort order": ("if (f[axis[j]] < f[axis[j + 1]])", "if (f[axis[j]] > f[axis[j + 1]])"),
    "tie rule": ("if (f[axis[j]] < f[axis[j + 1]])", "if (f[axis[j]] <= f[axis[j + 1]])"),
    "first weight": ("w64[0] = 1.0 - (double)f[axis[0]];", "w64[0] = 1.0 - (double)f[axis[n - 1]];"),
    "last weight": ("w64[n] = (double)f[axis[n - 1]];", "w64[n] = (double)f[axis[0]];"),
    "walk axis": ("verts[k][axis[k - 1]] += 1;", "verts[k][axis[n - k]] += 1;"),
    "hash prime": ("P[1] = 2654435761u;", "P[1] = 2654435769u;"),
    "hash op": ("h ^= (uint32_t)v[i] * g_primes[i];", "h += (uint32_t)v[i] * g_primes[i];"),
    "adjoint weight": ("d_tables[slot] += w64[k] * g;", "d_tables[slot] += g;"),
    "grid weight": ("w *= bit ? (double)f[i] : 1.0 - (double)f[i];",
                    "w *= bit ? 1.0 - (double)f[i] : (double)f[i];"),
    "mlp transposed": ("s += w * h1[i];", "s += orc_f16_to_f64(W2[i * H + o]) * h1[i];"),
    "mlp relu dropped": ("h2[o] = f16r(s > 0.0 ? s : 0.0);\n            a2[o] = s > 0.0 ? sa : 0.0;",
                         "h2[o] = f16r(s);\n            a2[o] = s > 0.0 ? sa : 0.0;"),
    "mlp bwd mask": ("dh1[i] = OP(h1[i] > 0.0 ? s : 0.0);", "dh1[i] = OP(s);"),
    "f16 rounding": ("double q = nearbyint(ldexp(a, 10 - e));", "double q = floor(ldexp(a, 10 - e));"),
    "mse sign": ("d_y[i] = scale * ((double)y[i] - (double)target[i]);",
                 "d_y[i] = scale * ((double)target[i] - (double)y[i]);"),
    "adam bias correction": ("double mhat = mi / bc1, vhat = vi / bc2;", "double mhat = mi, vhat = vi / bc2;"),
    "input grad skew chain": ("dx[m] += (double)sigma[l] * (g[m] + Fn * gs);", "dx[m] += (double)sigma[l] * g[m];"),
    "input grad walk difference": ("g[axis] += (t[k + 1][j] - t[k][j]) * d[j];", "g[axis] += (t[k][j] - t[k + 1][j]) * d[j];"),
    "input grad grid sign": ("double c = ((b >> i) & 1) ? 1.0 : -1.0;", "double c = 1.0;"),
    "composite own sample in transmittance": ("const double w = exp(-optical) * (-expm1(-tau));",
                                              "const double w = exp(-optical - tau) * (-expm1(-tau));"),
    "composite linear alpha": ("const double w = exp(-optical) * (-expm1(-tau));",
                               "const double w = exp(-optical) * tau;"),
    "composite density activation": ("const double sigma = softplus(q[0]);", "const double sigma = exp(q[0]);"),
    "composite adjoint remainder sign": ("dtau += dQ[ch] * (Tn * c[ch] - rest);",
                                         "dtau += dQ[ch] * (Tn * c[ch] + rest);"),
    "composite adjoint activation": ("const double ds = sigmoid(q[0]) * dl;", "const double ds = dl;"),
    # the magnitude outputs every GPU tolerance is scaled by
    "fwd magnitude drops the weight": ("acc += fabs(w64[k] * table_value(tables, e->table_dtype, row * F + j));",
                                       "acc += fabs(table_value(tables, e->table_dtype, row * F + j));"),
    "adjoint magnitude drops the weight": ("if (absmag) absmag[slot] += fabs(w64[k] * g);",
                                           "if (absmag) absmag[slot] += fabs(g);"),
    "input grad magnitude skew chain": ("ax[m] += (double)sigma[l] * (a[m] + Fn * as);",
                                        "ax[m] += (double)sigma[l] * a[m];"),
    "input grad magnitude sum of rows": ("a[axis] += fabs((t[k + 1][j] - t[k][j]) * d[j]);",
                                         "a[axis] += (fabs(t[k + 1][j]) + fabs(t[k][j])) * fabs(d[j]);"),
    "input grad grid magnitude factor": ("a[i] += fabs(c * t[b][j] * d[j]);", "a[i] += fabs(t[b][j] * d[j]);"),
    "mlp fwd magnitude unmasked": ("a1[o] = s > 0.0 ? sa : 0.0;", "a1[o] = sa;"),
    "mlp bwd magnitude unmasked": ("mh1[i] = h1[i] > 0.0 ? m : 0.0;", "mh1[i] = m;"),
    "mlp bwd magnitude dW3 factor": ("if (with_mag) mag_dW3[o * H + i] += fabs(dy[o]) * fabs(OP(h2[i]));",
                                     "if (with_mag) mag_dW3[o * H + i] += fabs(dy[o]);"),
    "mlp bwd exact mode rounds": ("#define OP(v) (mode == ORC_MLP_BF16 ? orc_round_bf16(v) : (v))",
                                  "#define OP(v) (orc_round_bf16(v))"),
    # the per-level table layout (Sec. 5.2)
    "dense row stride": ("            stride *= ext;\n", "            stride *= ext + 1;\n"),
    "dense clamp of negative coordinates": ("            if (c < 0) c = 0;\n", "\n"),
    "dense clamp of the upper face": ("            if (c > ext - 1) c = ext - 1;\n", "            if (c > ext) c = ext;\n"),
    "box extent one short": ("    return (int32_t)floorf(p) + 2;", "    return (int32_t)floorf(p) + 1;"),
    "used share exponent": ("for (int i = 0; i < n - 1; ++i) k *= (unsigned __int128)(n + 1);",
                            "for (int i = 0; i < n; ++i) k *= (unsigned __int128)(n + 1);"),
    "sized level offsets": ("        lay->off[l + 1] = lay->off[l] + rows;", "        lay->off[l + 1] = lay->off[l] + T;"),
    "composite magnitude remainder": ("atau += fabs(dQ[ch]) * (Tn * fabs(c[ch]) + fabs(Q[ch]) + fabs(part[ch]));",
                                      "atau += fabs(dQ[ch]) * (Tn * fabs(c[ch]) + fabs(Q[ch]));"),
}


def _run_mutant(name, old, new, tmp):
    src = open(SRC).read()
    assert src.count(old) >= 1, name
    path = os.path.join(tmp, name.replace(" ", "_") + ".c")
    lib = path[:-2] + ".so"
    open(path, "w").write(src.replace(old, new, 1))
    subprocess.run(["gcc", "-O1", "-std=c11", "-ffp-contract=off", "-fopenmp", "-fPIC", "-shared",
                    "-o", lib, path, "-lm"], check=True)
    env = dict(os.environ, SPX_ORACLE_LIB=lib, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return name, r.returncode


def test_every_planted_mistake_fails_a_pin():
    with tempfile.TemporaryDirectory() as tmp:
        with ThreadPoolExecutor(max_workers=max(1, min(8, os.cpu_count() or 1))) as ex:
            results = list(ex.map(lambda kv: _run_mutant(kv[0], *kv[1], tmp), MUTANTS.items()))
    survivors = [name for name, rc in results if rc == 0]
    assert not survivors, f"mutants not caught by the pins: {survivors}"
