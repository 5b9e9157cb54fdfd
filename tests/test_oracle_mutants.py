"""The narrow-arithmetic pins catch misplaced roundings.

Each case plants one plausible mistake in a copy of the oracle's source
(a rounding moved, added or dropped, an accumulation in the wrong
precision), compiles the copy into a temporary library and runs the pins of
test_oracle_narrow.py against it: at least one must fail.  The oracle
itself is not modified; the text replaced must occur exactly once."""
import os

import pytest

from oracle import build as OB
from tests import test_oracle_narrow as TN

SRC = os.path.join(os.path.dirname(OB.__file__), "f3r_oracle.c")

# (id, text in the oracle, replacement, pins that must catch it)
MUTANTS = [
    ("r: A z rounded to storage before v - A z",
     "r[i] = RND(p, RND(q, v[i] - t[i]));",
     "r[i] = RND(p, RND(q, v[i] - RND(p, t[i])));", "rich"),
    ("w': dots accumulated in the storage precision",
     "double num = ldot(h, q, n, r, t);\n      double den = ldot(h, q, n, t, t);",
     "double num = ldot(h, p, n, r, t);\n      double den = ldot(h, p, n, t, t);", "rich"),
    ("w': t = A y stored narrow instead of kept in fp32",
     "csr_mv(n, h->rp, h->ci, h->alev[L->pA], q, q, y, t);\n      h->st.spmv[d]++;\n      double num",
     "csr_mv(n, h->rp, h->ci, h->alev[L->pA], q, p, y, t);\n      h->st.spmv[d]++;\n      double num",
     "rich"),
    ("w': quotient rounded to the storage precision",
     "double wp = RND(q, num / den);", "double wp = RND(p, num / den);", "rich"),
    ("z update: w y rounded to storage before the sum",
     "z[i] = RND(p, RND(q, z[i] + RND(q, om[k] * y[i])));",
     "z[i] = RND(p, RND(q, z[i] + RND(p, om[k] * y[i])));", "rich"),
    ("weight mean divides by l instead of l + 1",
     "/ (double)(l + 1));", "/ (double)(l > 1 ? l : 2));", "rich"),
    ("R input not rounded to the level storage",
     "for (int64_t i = 0; i < n; i++) v[i] = RND(p, vin[i]);\n  OR_PAR_FOR\n  for (int64_t i = 0; i < n; i++) z[i] = 0.0;",
     "for (int64_t i = 0; i < n; i++) v[i] = vin[i];\n  OR_PAR_FOR\n  for (int64_t i = 0; i < n; i++) z[i] = 0.0;",
     "rich"),
    ("M: intermediate W r not rounded to storage",
     "csr_mv(h->n, h->wrp, h->wci, wv, q, pv, r, h->mtmp);",
     "csr_mv(h->n, h->wrp, h->wci, wv, q, q, r, h->mtmp);", "rich"),
    ("M: sums accumulated in the storage precision",
     "csr_mv(h->n, h->grp, h->gci, gv, q, pv, h->mtmp, y);",
     "csr_mv(h->n, h->grp, h->gci, gv, pv, pv, h->mtmp, y);", "rich"),
    ("FGMRES: orthogonalised w stored in fp16",
     "w[k] = RND(p, acc);", "w[k] = RND(p == OR_F32 ? OR_F16 : p, acc);", "fgmres"),
    ("FGMRES: level SpMV accumulated in the matrix precision",
     "csr_mv(n, h->rp, h->ci, h->alev[L->pA], q, p, Zc(j), w);",
     "csr_mv(n, h->rp, h->ci, h->alev[L->pA], L->pA, p, Zc(j), w);", "fgmres"),
    ("FGMRES: Givens update of g in fp16",
     "W->g[j + 1] = RND(q, -W->sn[j] * W->g[j]);",
     "W->g[j + 1] = RND(q == OR_F32 ? OR_F16 : q, -W->sn[j] * W->g[j]);", "fgmres"),
    ("FGMRES: back substitution in fp16",
     "W->y[i] = RND(q, acc / Hh(i, i));",
     "W->y[i] = RND(q == OR_F32 ? OR_F16 : q, acc / Hh(i, i));", "fgmres"),
    ("FGMRES: dots h_ij rounded to fp16",
     "for (int i = 0; i <= j; i++) Hh(i, j) = ldot(h, q, n, w, Vc(i));",
     "for (int i = 0; i <= j; i++) Hh(i, j) = RND(q == OR_F32 ? OR_F16 : q, ldot(h, q, n, w, Vc(i)));",
     "fgmres"),
    ("FGMRES: norm h_{j+1,j} rounded to fp16",
     "static double lnrm2(const or_handle* h, int32_t q, int64_t n, const double* x) {\n  return RND(q, sqrt(ldot(h, q, n, x, x)));",
     "static double lnrm2(const or_handle* h, int32_t q, int64_t n, const double* x) {\n  return RND(q == OR_F32 ? OR_F16 : q, sqrt(ldot(h, q, n, x, x)));",
     "fgmres"),
    ("FGMRES: output Z y summed in fp16",
     "for (int j = 0; j < meff; j++) acc = RND(q, acc + RND(q, W->y[j] * Zc(j)[k]));",
     "for (int j = 0; j < meff; j++) acc = RND(q == OR_F32 ? OR_F16 : q, acc + RND(q, W->y[j] * Zc(j)[k]));",
     "fgmres"),
]


@pytest.mark.parametrize("mid,old,new,which", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, mid, old, new, which):
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site not found once: {old!r}"
    mut = tmp_path / "mutant.c"
    mut.write_text(src.replace(old, new))
    lib = OB.build(src=str(mut), out=str(tmp_path / "libmutant.so"))
    run = TN.run_richardson_pins if which == "rich" else TN.run_fgmres32_pins
    with pytest.raises(AssertionError):
        run(lib_path=lib)
