"""The oracle's pins catch planted mistakes.

Each case copies the oracle's C source, plants one plausible mistake (a wrong
sign, a dropped term, an off-by-one, a wrong index or level), builds the copy
with gcc and runs the oracle pin tests against it in a child process.  The
case passes when at least one pin fails: a mistake that every pin accepts
would be a hole in the oracle's checks.  Nothing here touches the GPU or the
HIP library; the mistakes are planted in a temporary copy of the oracle only.
"""
import concurrent.futures
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "treecode_oracle.c")
PINS = ["tests/test_oracle_keys_tree.py", "tests/test_oracle_forces.py", "tests/test_oracle_adjoint.py"]

# (name, text in the oracle, planted replacement, occurrences replaced)
MUTANTS = [
    # root cube and keys (O2-O4)
    ("root-cube-not-smallest-power", "int eL = (f == 0.5) ? e - 1 : e;", "int eL = e;", 1),
    ("quantise-rounds", "double f = floor(scaled);", "double f = nearbyint(scaled);", 1),
    ("clamp-one-too-high", "#define OR_QMAX ((int64_t)(1 << 21) - 1)", "#define OR_QMAX ((int64_t)(1 << 21))", 1),
    ("interleave-y-high", "<< (3 * b + 2);\n        key |= (uint64_t)((qy >> b) & 1) << (3 * b + 1);",
     "<< (3 * b + 1);\n        key |= (uint64_t)((qy >> b) & 1) << (3 * b + 2);", 1),
    ("sort-unstable-on-ties", "if (keys[src[j]] < keys[src[i]])", "if (keys[src[j]] <= keys[src[i]])", 1),
    # topology (O6)
    ("leaf-at-level-20", "if (e - b == 1 || level == OR_MAXLEVEL) return id;",
     "if (e - b == 1 || level == OR_MAXLEVEL - 1) return id;", 1),
    ("digit-from-shifted-triple", "return (int)((key >> (3 * (OR_MAXLEVEL - level))) & 7u);",
     "return (int)((key >> (3 * (OR_MAXLEVEL - level) + 1)) & 7u);", 1),
    # moments (O7)
    ("com-not-divided-by-mass", "for (int k = 0; k < 3; ++k) T->com[3 * id + k] = S[k] / M;",
     "for (int k = 0; k < 3; ++k) T->com[3 * id + k] = S[k];", 1),
    ("child-com-unweighted", "S[k] += T->mass[ch] * T->com[3 * ch + k];", "S[k] += T->com[3 * ch + k];", 1),
    ("leaf-mass-skips-first", "            for (int64_t j = b; j < e; ++j) {\n                M += T->sm[j];",
     "            for (int64_t j = b + 1; j < e; ++j) {\n                M += T->sm[j];", 1),
    # walk (O8) and the interaction (Eq.(1))
    ("containment-rule-dropped", "    int contains = (si >= b && si < e);\n    if (contains) {",
     "    int contains = 0;\n    if (contains) {", 1),
    ("criterion-side-of-child-level", "double side = ldexp(T->L, -T->level[id]);\n    if (C->theta",
     "double side = ldexp(T->L, -T->level[id] - 1);\n    if (C->theta", 1),
    ("criterion-squared-distance", "if (C->theta > 0.0 && side < C->theta * dist)",
     "if (C->theta > 0.0 && side < C->theta * dist * dist)", 1),
    ("self-term-in-own-leaf", "                if (j != si) term(r, x, &T->sx[3 * j], T->sm[j], C->eps2, C->G);",
     "                term(r, x, &T->sx[3 * j], T->sm[j], C->eps2, C->G);", 1),
    ("force-sign", "r->a[k] += G * mu * d[k] * inv3;", "r->a[k] -= G * mu * d[k] * inv3;", 1),
    ("softening-eps-not-squared", "J.C.eps2 = eps * eps;", "J.C.eps2 = eps;", 1),
    ("potential-power", "r->phi -= G * mu * inv;", "r->phi -= G * mu * inv * inv;", 1),
    ("direct-sum-includes-self", "        if (j != i) term(&r, &J->pos[3 * i], &J->pos[3 * j], J->m[j], J->eps2, J->G);",
     "        term(&r, &J->pos[3 * i], &J->pos[3 * j], J->m[j], J->eps2, J->G);", 1),
    # frozen lists and the adjoint
    ("frozen-moments-ignore-new-masses", "        sm[s] = m[i];", "        sm[s] = T->sm[s];", 1),
    ("adjoint-tensor-sign", "- 3.0 * inv5 * d[k] * dg", "+ 3.0 * inv5 * d[k] * dg", 1),
    ("adjoint-mass-term-sign", "gmu = G * (dg * inv3 - h * inv);", "gmu = G * (dg * inv3 + h * inv);", 1),
    ("adjoint-no-prefix-sum", "U[3 * id + k] = (p >= 0 ? U[3 * p + k] : 0.0) + u[k];", "U[3 * id + k] = u[k];", 1),
    ("adjoint-offset-sign", "cc = gM[id] - (", "cc = gM[id] + (", 1),
    ("adjoint-target-side-dropped", "for (int k = 0; k < 3; ++k) gx[3 * si + k] -= gy[k];", "", 1),
    # leapfrog, Eqs.(2)-(5)
    ("leapfrog-full-first-kick", "for (int64_t i = 0; i < 3 * n; ++i) vel[i] += 0.5 * tau * acc[i];\n    for (int64_t i = 0; i < 3 * n; ++i) pos[i]",
     "for (int64_t i = 0; i < 3 * n; ++i) vel[i] += tau * acc[i];\n    for (int64_t i = 0; i < 3 * n; ++i) pos[i]", 1),
    ("leapfrog-drift-half-step", "pos[i] += tau * vel[i];", "pos[i] += 0.5 * tau * vel[i];", 1),
]

CFLAGS = ["-O3", "-fno-fast-math", "-ffp-contract=off", "-fPIC", "-shared", "-std=c11", "-pthread"]


def _run_mutant(tmpdir, name, old, new, count):
    src = open(SRC).read()
    found = src.count(old)
    if found != count:
        return name, "the text to mutate occurs %d times, expected %d" % (found, count)
    d = os.path.join(tmpdir, name)
    os.makedirs(d, exist_ok=True)
    c = os.path.join(d, "oracle_mutant.c")
    so = os.path.join(d, "liboracle_mutant.so")
    with open(c, "w") as f:
        f.write(src.replace(old, new))
    r = subprocess.run(["gcc", *CFLAGS, "-o", so, c, "-lm"], capture_output=True, text=True)
    if r.returncode != 0:
        return name, "mutant does not compile: " + r.stderr[-400:]
    env = dict(os.environ, TREECODE_ORACLE_LIB=so, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PINS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # pytest exit code 1: some test failed (the mistake was caught)
    if r.returncode == 1:
        return name, None
    if r.returncode == 0:
        return name, "every pin passed with the mistake planted"
    return name, "pytest ended with code %d: %s" % (r.returncode, r.stdout[-400:])


def test_mutant_texts_are_unique():
    names = [m[0] for m in MUTANTS]
    assert len(names) == len(set(names))
    src = open(SRC).read()
    for name, old, new, count in MUTANTS:
        assert src.count(old) == count, name
        assert old != new, name


def test_pins_catch_every_planted_mistake(tmp_path):
    workers = max(1, min(4, (os.cpu_count() or 2) // 2))
    with concurrent.futures.ThreadPoolExecutor(max_workers=workers) as ex:
        futs = [ex.submit(_run_mutant, str(tmp_path), *m) for m in MUTANTS]
        results = [f.result() for f in futs]
    missed = ["%s: %s" % (n, why) for n, why in results if why is not None]
    assert not missed, "\n".join(missed)
