"""Planted mistakes: each plausible error, planted in a copy of the oracle on
the CPU, must make at least one pin fail.  This checks that the pins pin the
oracle (a dropped term, a wrong sign or index, a transposed operand, a wrong
threshold or order), not that the oracle is right."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

F = "tests/test_oracle_forward.py"
B = "tests/test_oracle_backward.py"
N = "tests/test_oracle_bin.py"
V = "tests/test_oracle_variants.py"
C = "tests/test_oracle_cull.py"

MUTANTS = [
    ("camera matrix uses W instead of W-1", "out[0] = -((double)W - 1.0) / fov_h;", "out[0] = -((double)W) / fov_h;", [F]),
    ("h_y = v x h_x", "cross3(hx, v, hy);", "cross3(v, hx, hy);", [F]),
    ("near test sign", "if (!(t > near_m)) return 0;", "if (!(t > -near_m)) return 0;", [F]),
    ("support 2.5 sigma", "#define OR_SUPPORT 3.0", "#define OR_SUPPORT 2.5", [F]),
    ("support 3.5 sigma", "#define OR_SUPPORT 3.0", "#define OR_SUPPORT 3.5", [F]),
    ("contributors sorted far to near", "if (x->key < y->key) return -1;", "if (x->key > y->key) return -1;", [F]),
    ("transmittance update halves alpha", "T *= 1.0 - p->alpha;", "T *= 1.0 - 0.5 * p->alpha;", [F]),
    ("A_k off by one", "double A = Apre[c], a", "double A = Apre[c + 1], a", [B]),
    ("opacity channel dropped", "dA += gO * Tfin / om;", "dA += 0.0 * gO * Tfin / om;", [B]),
    ("alpha clamp ignored in the gradient", "if (!p->clamped) { gs[0]", "if (1) { gs[0]", [B]),
    ("rho_beta sign", "gA[k] = -rb[0] * hx[k]", "gA[k] = rb[0] * hx[k]", [B]),
    ("dR/dx entry", "double dRx[9] = {0, 2 * y, 2 * z,", "double dRx[9] = {0, 2 * z, 2 * y,", [B]),
    ("pose translation sign", "gpose[c] -= g[6 + c];", "gpose[c] += g[6 + c];", [B]),
    ("pose rotation drops the normal term", "t1[c] + t2[c] + t3[c] + t4[c]", "t1[c] + t2[c] + t3[c]", [B]),
    ("box without edge stationary points", "if (ts > 0.0 && ts < 1.0) {", "if (0) {", [N]),
    ("box margin rotated the wrong way",
     "double lx = V[klo][0] * T->cm + V[klo][1] * T->sm, ly = V[klo][1] * T->cm - V[klo][0] * T->sm;",
     "double lx = V[klo][0] * T->cm - 200.0 * V[klo][1] * T->sm, ly = V[klo][1] * T->cm + 200.0 * V[klo][0] * T->sm;",
     [N]),
    ("variants never branch on the stop rule", "} else if (fabs(tT - OR_T_MIN) < c->gT * OR_T_MIN) {",
     "} else if (0) {", [V]),
    ("variants ignore the alpha-floor band", "fam = fabs(a - OR_ALPHA_MIN) < guard[2] * OR_ALPHA_MIN;", "fam = 0;", [V]),
    ("variant branch keeps the inclusion", "vwalk(c, i, T, D, N, O, flips + 1, !inc, -1);",
     "vwalk(c, i, T, D, N, O, flips + 1, inc, -1);", [V]),
    ("cull sphere radius without the 3-sigma factor",
     "double r = 3.0 * sqrt(F[k].s[0] * F[k].s[0] + F[k].s[1] * F[k].s[1]) * 1.001 + 1e-9;",
     "double r = sqrt(F[k].s[0] * F[k].s[0] + F[k].s[1] * F[k].s[1]) * 1.001 + 1e-9;", [C]),
    ("cull tests only the forward half of the line",
     "if (fabs(v[0] * c[0] + v[1] * c[1] + v[2] * c[2]) < c[3]) continue;\n            or_pair p;",
     "if ((v[0] * c[0] + v[1] * c[1] + v[2] * c[2]) < c[3]) continue;\n            or_pair p;", [C]),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,old,new,targets", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, name, old, new, targets):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not unique: {old}"
    c = tmp_path / "oracle_mut.c"
    c.write_text(src.replace(old, new))
    so = tmp_path / "liboracle_mut.so"
    subprocess.run(["gcc", "-O1", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-shared", "-fPIC",
                    str(c), "-o", str(so), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(so), OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "4"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        *targets], cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    assert r.returncode == 1, f"pins did not catch the planted mistake '{name}':\n{r.stdout[-2000:]}"
