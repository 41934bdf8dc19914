"""Planted mistakes: every mutant of the oracle must fail the oracle's pins.

Each entry plants one plausible slip in one step of oracle/oracle.c (a wrong
constant, a dropped term, a transposed operand, an off-by-one, a sign) in a
copy of the source, builds it, and runs tests/test_oracle.py against that
build in a child process (ORACLE_LIB).  The pins must fail for every mutant:
they check the oracle against what the paper and the mathematics fix, so a
mistake anywhere in it shows.  The unmodified source must pass the same run.
CPU only; the child runs skip the rocRAND cross-check, which compiles a helper
(the known-answer vectors pin the generator)."""
from __future__ import annotations

import concurrent.futures as cf
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

# (name, text in oracle.c, replacement)
MUTANTS = [
    ("philox multiplier", "uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;",
     "uint64_t p0 = (uint64_t)0xD2511F52u * (uint64_t)c0;"),
    ("philox key increment", "k1 += 0xBB67AE85u;", "k1 += 0xBB67AE84u;"),
    ("philox output order", "out[0] = c0; out[1] = c1;", "out[0] = c1; out[1] = c0;"),
    ("uniform from the low word only", "return ((uint64_t)o0 << 21) | ((uint64_t)o1 >> 11);",
     "return ((uint64_t)o1 >> 11);"),
    ("holding time scaled by the rate", "S = -log(uniform_open0(rnd[0], rnd[1])) * ts->inv_r[x];",
     "S = -log(uniform_open0(rnd[0], rnd[1])) * ts->r[x];"),
    ("jump test forgets elapsed time", "jump = s + S < o->t;", "jump = S < o->t;"),
    ("slot index misses the last slot",
     "(((uint64_t)rnd[2] * (uint64_t)ts->deg[x]) >> 32)",
     "(((uint64_t)rnd[2] * (uint64_t)(ts->deg[x] - 1)) >> 32)"),
    ("alias column of the wrong slot", "alias[s] = col[alias_slot[s]];", "alias[s] = col[s];"),
    ("vose update", "q[g] = (q[g] + q[l]) - 1.0;", "q[g] = q[g] - q[l];"),
    ("alias test reversed", "if (rnd[3] < ts->thr[q]) {", "if (rnd[3] >= ts->thr[q]) {"),
    ("scaled probability without deg", "q[s] = (ts->val[b + s] * (double)deg) / rate;",
     "q[s] = ts->val[b + s] / rate;"),
    ("weight exponent drops the diagonal", "ts->d[i] = diag + rate;", "ts->d[i] = rate;"),
    ("weight exponent drops the rate", "ts->d[i] = diag + rate;", "ts->d[i] = diag;"),
    ("exact weight uses the jump time", "logw += ts->d[path_x[m]] * held;",
     "logw += ts->d[path_x[m]] * sb;"),
    ("last holding interval dropped",
     "double held = (m < len) ? (sb - path_s[m]) : (o->t - path_s[m]);",
     "double held = (m < len) ? (sb - path_s[m]) : 0.0;"),
    ("trapezoid end weights", "return (k == 0 || k == o->ngrid) ? 0.5 : 1.0;", "return 1.0;"),
    ("right Riemann sum includes k = 0", "return k == 0 ? 0.0 : 1.0;", "return 1.0;"),
    ("grid index rounds down", "double g = ceil(s * o->inv_dt);", "double g = floor(s * o->inv_dt);"),
    ("value read at the start node", "res->f = exp(logw) * v[x];", "res->f = exp(logw) * v[start];"),
    ("tilt correction sign", "ts->logcorr[slot] = -(double)bias[p];",
     "ts->logcorr[slot] = (double)bias[p];"),
    ("tilted exponent not shifted", "ts->d[i] = base->d[i] + (rate - base->r[i]);",
     "ts->d[i] = base->d[i];"),
    ("alias jump takes its own correction",
     "corr = ts->logcorr[ts->begin[x] + ts->alias_slot[q]];", "corr = ts->logcorr[q];"),
    ("mean over M + 1", "double mean = neumaier_sum(fs, jb->nwalk) / (double)jb->nwalk;",
     "double mean = neumaier_sum(fs, jb->nwalk) / (double)(jb->nwalk + 1);"),
    ("standard error without 1/M", "jb->se[e] = sqrt(var / (double)jb->nwalk);",
     "jb->se[e] = sqrt(var);"),
    ("variance from the raw second moment", "dev[w] = (fs[w] - mean) * (fs[w] - mean);",
     "dev[w] = fs[w] * fs[w];"),
    ("negative rates accepted", "else if (col[p] != i && val[p] < 0.0) bad_sign = 1;",
     "else if (col[p] != i && val[p] < -1.0) bad_sign = 1;"),
    ("forward starts weighted by v, not |v|", "V = V + fabs(v[j]);", "V = V + v[j];"),
    ("forward value without the sign", "y = V * (v[lo] > 0.0 ? 1.0 : -1.0) * exp(r.logw);",
     "y = V * exp(r.logw);"),
    ("forward value credited to the start", "x_end = r.x_end;", "x_end = (int32_t)lo;"),
    ("conditioned first time not truncated",
     "S = -log(1.0 - uniform_open1(rnd[0], rnd[1]) * q) * ts->inv_r[x];",
     "S = -log(uniform_open0(rnd[0], rnd[1])) * ts->inv_r[x];"),
    ("conditioned value without the no-jump term",
     "res->f = exp(-rt) * (exp(logk) * v[start]) + (-expm1(-rt)) * res->f;",
     "res->f = (-expm1(-rt)) * res->f;"),
    ("conditioned value without the jump probability",
     "res->f = exp(-rt) * (exp(logk) * v[start]) + (-expm1(-rt)) * res->f;",
     "res->f = exp(-rt) * (exp(logk) * v[start]) + res->f;"),
    ("lattice points not spread over the replicate",
     "const uint64_t u0 = (j << (64 - b)) + (((uint64_t)sh[0] << 32) | sh[1]);",
     "const uint64_t u0 = (j << (63 - b)) + (((uint64_t)sh[0] << 32) | sh[1]);"),
    ("lattice points in ordinal order, not radical-inverse",
     "const uint64_t j = radical_index(w & ((1u << b) - 1u), b);",
     "const uint64_t j = w & ((1u << b) - 1u);"),
    ("lattice shift shared by every replicate",
     "uint32_t ctr[4] = { QMC_SHIFT_MARK, w >> b, (uint32_t)start, o->instance };",
     "uint32_t ctr[4] = { QMC_SHIFT_MARK, 0u, (uint32_t)start, o->instance };"),
    ("lattice slot word without the lattice point",
     "rnd[2] = (uint32_t)(((j * g1) << (32 - b)) + sh[2]);", "rnd[2] = sh[2];"),
    ("replicate error without R/(R-1)",
     "jb->se[e] = sqrt(acc * (double)R / (double)(R - 1));", "jb->se[e] = sqrt(acc);"),
    ("inverse-CDF target not scaled by the rate",
     "const double target = ((double)rnd[2] * 0x1p-32) * ts->r[x];",
     "const double target = ((double)rnd[2] * 0x1p-32);"),
    ("inverse-CDF takes the slot after the crossing", "if (target < cum) { sl = k; break; }",
     "if (target < cum) { sl = k + 1 < ts->deg[x] ? k + 1 : k; break; }"),
    ("forward grid not reversed",
     "acc += grid_coef(o, forward ? o->ngrid - k : k) * ts->d[path_x[m]];",
     "acc += grid_coef(o, k) * ts->d[path_x[m]];"),
]


def _build(tmp, name, text):
    c = os.path.join(tmp, name + ".c")
    so = os.path.join(tmp, name + ".so")
    open(c, "w").write(text)
    subprocess.run(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC",
                    "-shared", "-pthread", c, "-o", so, "-lm"], check=True,
                   capture_output=True)
    return so


def _run_pins(so):
    env = dict(os.environ, ORACLE_LIB=so)
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle.py"),
                        "-x", "-q", "-p", "no:cacheprovider", "--timeout", "60",
                        "-k", "not rocrand"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    failed = re.findall(r"FAILED (\S+)", r.stdout)
    return r.returncode, failed[0] if failed else r.stdout[-300:]


@pytest.fixture(scope="module")
def outcomes(tmp_path_factory):
    tmp = str(tmp_path_factory.mktemp("mutants"))
    src = open(SRC).read()
    jobs = {"unmodified": _build(tmp, "unmodified", src)}
    for k, (name, old, new) in enumerate(MUTANTS):
        assert src.count(old) == 1, f"mutant {name!r}: text not found exactly once"
        jobs[name] = _build(tmp, f"m{k}", src.replace(old, new))
    with cf.ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        futs = {name: ex.submit(_run_pins, so) for name, so in jobs.items()}
        return {name: f.result() for name, f in futs.items()}


def test_unmodified_oracle_passes(outcomes):
    rc, info = outcomes["unmodified"]
    assert rc == 0, info


@pytest.mark.parametrize("name", [m[0] for m in MUTANTS])
def test_mutant_is_caught(outcomes, name):
    rc, info = outcomes[name]
    # exit status 1: a pin failed (not a crash or a collection error)
    assert rc == 1, f"mutant {name!r} survived or crashed (rc={rc}): {info}"
