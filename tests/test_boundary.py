"""The boundary between the Python binding and the C-ABI library (CPU only).

* Every function the binding declares argument types for has the same number
  of parameters in include/msqd.h, so no call passes or drops an argument.
* The readouts the boundary promises are declared with their outputs:
  dipole_readout's FP64 ensemble sums, the <R>_e ratio of excited_r_readout,
  the T/R/A spectra of spectra_readout.
* The binding does no arithmetic on what the library returns: no division,
  no reductions (sum, mean, norm, ...) and no elementwise math in msqd.py.
  The only arithmetic left there is integer bookkeeping of buffer sizes and
  step counters.
"""

import ast
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "msqd.h")
BINDING = os.path.join(ROOT, "paper_2209_04487_amd", "msqd.py")


def _declarations():
    """name -> list of parameter strings, from the header without comments."""
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    out = {}
    for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s+([a-z_][a-z0-9_]*)\s*\(([^;]*?)\)\s*;",
                         text, flags=re.M | re.S):
        params = " ".join(m.group(2).split())
        out[m.group(1)] = [] if params in ("", "void") else [p.strip() for p in params.split(",")]
    return out


def test_binding_argument_counts_match_the_header():
    from paper_2209_04487_amd import msqd
    decl = _declarations()
    for name, (_res, args) in msqd._sigs.items():
        assert name in decl, name
        assert len(args) == len(decl[name]), (name, len(args), decl[name])
    # and the binding covers every declared entry point
    assert set(decl) == set(msqd._sigs), set(decl) ^ set(msqd._sigs)


def test_readouts_declared_with_their_outputs():
    decl = _declarations()
    assert decl["dipole_readout"][-2] == "double* sums"
    assert decl["excited_r_readout"][-2] == "double* sums"
    text = open(HEADER).read()
    assert "sums: device\n * float64 [3] = (sum r_num, sum pop, their ratio" in text
    assert decl["spectra_readout"] == ["const fdtd_desc* d", "const double* flux", "const double* flux_ref",
                                       "double* tra", "void* stream"]


_REDUCTIONS = {"sum", "mean", "prod", "norm", "std", "var", "abs", "sqrt", "exp", "cumsum", "dot",
               "matmul", "einsum", "max", "min", "real", "imag"}


def test_binding_does_no_arithmetic_on_results():
    tree = ast.parse(open(BINDING).read())
    bad = []
    for node in ast.walk(tree):
        if isinstance(node, ast.BinOp) and isinstance(node.op, (ast.Div, ast.Pow, ast.MatMult)):
            bad.append((node.lineno, type(node.op).__name__))
        if isinstance(node, ast.Call) and isinstance(node.func, ast.Attribute) and node.func.attr in _REDUCTIONS:
            bad.append((node.lineno, node.func.attr))
    assert not bad, bad
