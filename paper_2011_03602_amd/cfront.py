"""C programs on the same boundary: a front end for a subset of C99.

The paper's analysis is common to every language; only the parsing is
per language (Sec. 4.3). This module is the C parser. It tokenizes and parses
one C function and lowers it into the representation the Python front end
analyses, a Python function with the same loops, subscripts and assignments.
The shared analysis then runs unchanged: loop statements, the offload screen,
variable sets, binding by what the nests compute, plans through
ofl_plan_nests, and runs through the loop gene.

The subset:

- One function. Its parameters are ``int``/``float`` scalars and arrays
  declared with variable-length dimensions, e.g. ``float p[nz][ny][nx]``;
  ``const`` marks read-only arrays.
- A body of declarations, assignments (``=``, ``+=``), ``for`` loops over
  ``int`` counters (``for (int k = a; k < b; ++k)``, ``<=`` also), blocks and
  one final ``return``.
- Expressions with ``+ - * /``, unary minus, parentheses, numbers (a ``f``
  suffix is allowed), names and subscripts.

Lowering:

- The dimension parameters of the first array become its shape, unpacked at the
  top of the function.
- Local arrays (scratch) become extra inputs the driver supplies zero-filled.
- Non-const array parameters the function writes are visible to the caller
  after the call, so they join the values it returns.

``run_c`` compiles the program with gcc and runs it on numpy arrays: the
original program the offloaded runs are checked against.
"""

from __future__ import annotations

import ctypes
import os
import re
import subprocess
import tempfile
import threading
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import frontend as fe
from .frontend import FrontendError

_TOKEN = re.compile(r"""
    (?P<ws>\s+|//[^\n]*|/\*.*?\*/)
  | (?P<num>(\d+\.\d*|\.\d+|\d+)([eE][+-]?\d+)?[fF]?)
  | (?P<id>[A-Za-z_]\w*)
  | (?P<op>\+\+|--|\+=|-=|\*=|/=|<=|>=|==|!=|[-+*/=<>;,(){}\[\]])
""", re.X | re.S)

_TYPES = ("int", "float", "double", "void")


def tokenize(src: str) -> List[Tuple[str, str, int]]:
    out, pos, line = [], 0, 1
    while pos < len(src):
        m = _TOKEN.match(src, pos)
        if not m:
            raise FrontendError(f"C line {line}: cannot read {src[pos:pos + 20]!r}")
        kind = m.lastgroup
        text = m.group(kind)
        if kind != "ws":
            out.append((kind, text, line))
        line += text.count("\n")
        pos = m.end()
    return out


@dataclass
class Param:
    name: str
    ctype: str
    dims: List[str] = field(default_factory=list)   # C source of each dimension (arrays)
    const: bool = False


@dataclass
class CProgram:
    """What the C parser read, and the Python function it lowers to."""

    source: str
    func: str
    params: List[Param]
    local_arrays: Dict[str, List[str]]
    written: List[str]
    python: str
    rtype: str = "float"
    program: Optional[fe.Program] = None


class _Parser:
    def __init__(self, toks):
        self.t = toks
        self.i = 0

    def peek(self, k=0):
        return self.t[self.i + k] if self.i + k < len(self.t) else ("eof", "", -1)

    def take(self, text=None):
        tok = self.peek()
        if text is not None and tok[1] != text:
            raise FrontendError(f"C line {tok[2]}: expected {text!r}, found {tok[1]!r}")
        self.i += 1
        return tok

    def accept(self, text):
        if self.peek()[1] == text:
            self.i += 1
            return True
        return False

    # expressions, as Python source text
    def expr(self):
        left = self.term()
        while self.peek()[1] in ("+", "-"):
            op = self.take()[1]
            left = f"{left} {op} {self.term()}"
        return left

    def term(self):
        left = self.unary()
        while self.peek()[1] in ("*", "/"):
            op = self.take()[1]
            left = f"{left} {op} {self.unary()}"
        return left

    def unary(self):
        if self.accept("-"):
            return f"-{self.unary()}"
        if self.accept("+"):
            return self.unary()
        return self.primary()

    def primary(self):
        kind, text, line = self.peek()
        if text == "(":
            self.take("(")
            e = self.expr()
            self.take(")")
            return f"({e})"
        if kind == "num":
            self.take()
            return text.rstrip("fF")
        if kind == "id":
            self.take()
            if self.peek()[1] == "[":
                idx = []
                while self.accept("["):
                    idx.append(self.expr())
                    self.take("]")
                return f"{text}[{', '.join(idx)}]"
            if self.peek()[1] == "(":
                raise FrontendError(f"C line {line}: function calls are not read by the front end")
            return text
        raise FrontendError(f"C line {line}: unexpected {text!r} in an expression")

    def lvalue(self):
        kind, text, line = self.take()
        if kind != "id":
            raise FrontendError(f"C line {line}: expected a name to assign")
        idx = []
        while self.accept("["):
            idx.append(self.expr())
            self.take("]")
        return text, idx


def _parse_function(toks) -> Tuple[str, str, List[Param], list]:
    p = _Parser(toks)
    kind, rtype, line = p.take()
    if rtype not in _TYPES:
        raise FrontendError(f"C line {line}: expected a return type")
    name = p.take()[1]
    p.take("(")
    params: List[Param] = []
    while not p.accept(")"):
        const = p.accept("const")
        ctype = p.take()[1]
        if ctype not in _TYPES:
            raise FrontendError(f"C line {p.peek()[2]}: parameter type {ctype!r} is not read")
        pname = p.take()[1]
        dims = []
        while p.accept("["):
            dims.append(p.expr())
            p.take("]")
        params.append(Param(pname, ctype, dims, const))
        p.accept(",")
    p.take("{")
    body = _block(p)
    if p.peek()[0] != "eof":
        raise FrontendError("C: only one function is read")
    return rtype, name, params, body


def _block(p: _Parser) -> list:
    """Statements up to the matching '}' (already past the '{')."""
    out = []
    while not p.accept("}"):
        out.append(_stmt(p))
    return out


def _stmt(p: _Parser):
    kind, text, line = p.peek()
    if text == "{":
        p.take("{")
        return ("block", _block(p))
    if text == "for":
        p.take("for")
        p.take("(")
        p.take("int")
        var = p.take()[1]
        p.take("=")
        lo = p.expr()
        p.take(";")
        if p.take()[1] != var:
            raise FrontendError(f"C line {line}: the loop test must name the counter")
        cmp = p.take()[1]
        hi = p.expr()
        p.take(";")
        step = [p.take()[1] for _ in range(2)]
        if step not in (["++", var], [var, "++"]):
            raise FrontendError(f"C line {line}: loops must step with ++")
        p.take(")")
        if cmp == "<=":
            hi = f"{hi} + 1"
        elif cmp != "<":
            raise FrontendError(f"C line {line}: loop tests are < or <=")
        return ("for", var, lo, hi, _stmt(p), line)
    if text in ("while", "do", "if", "switch", "goto", "break", "continue"):
        raise FrontendError(f"C line {line}: {text} is not read by the front end")
    if text == "return":
        p.take("return")
        e = p.expr()
        p.take(";")
        return ("return", e)
    if text in ("float", "int", "double", "const"):
        p.accept("const")
        p.take()
        name = p.take()[1]
        dims = []
        while p.accept("["):
            dims.append(p.expr())
            p.take("]")
        init = None
        if p.accept("="):
            init = p.expr()
        p.take(";")
        return ("decl", name, dims, init)
    name, idx = p.lvalue()
    op = p.take()[1]
    if op not in ("=", "+="):
        raise FrontendError(f"C line {line}: assignments are = or +=")
    e = p.expr()
    p.take(";")
    return ("assign", name, idx, op, e)


def _lower(name: str, params: List[Param], body: list) -> Tuple[str, Dict[str, List[str]], List[str]]:
    arrays = [q for q in params if q.dims]
    if not arrays:
        raise FrontendError("C: the function takes no arrays")
    shape = arrays[0].dims
    for q in arrays:
        if q.dims != shape:
            raise FrontendError(f"C: array {q.name} is not shaped like {arrays[0].name}")
    dim_names = set(shape)
    local_arrays: Dict[str, List[str]] = {}
    written: List[str] = []
    lines: List[str] = []
    ret = None

    def emit(stmts, indent):
        nonlocal ret
        pad = "    " * indent
        for s in stmts:
            if s[0] == "block":
                emit(s[1], indent)
            elif s[0] == "for":
                _, var, lo, hi, inner, _line = s
                lines.append(f"{pad}for {var} in range({lo}, {hi}):")
                before = len(lines)
                emit([inner], indent + 1)
                if len(lines) == before:
                    lines.append(f"{pad}    pass")
            elif s[0] == "decl":
                _, nm, dims, init = s
                if dims:
                    if dims != shape:
                        raise FrontendError(f"C: local array {nm} is not shaped like the parameters")
                    local_arrays[nm] = dims
                elif init is not None:
                    lines.append(f"{pad}{nm} = {init}")
            elif s[0] == "assign":
                _, nm, idx, op, e = s
                target = f"{nm}[{', '.join(idx)}]" if idx else nm
                lines.append(f"{pad}{target} {op} {e}")
                if idx and nm not in written:
                    written.append(nm)
            elif s[0] == "return":
                if indent != 1:
                    raise FrontendError("C: return only at the end of the function")
                ret = s[1]
    emit(body, 1)
    visible = [q.name for q in arrays if not q.const and q.name in written]
    consts = [q.name for q in arrays if q.const and q.name in written]
    if consts:
        raise FrontendError(f"C: const arrays written: {consts}")
    outs = ([ret] if ret else []) + visible
    scalars = [q.name for q in params if not q.dims and q.name not in dim_names]
    py_params = [q.name for q in arrays] + list(local_arrays) + scalars
    head = [f"def {name}({', '.join(py_params)}):", f"    {', '.join(shape)} = {arrays[0].name}.shape"]
    tail = [f"    return {', '.join(outs)}"] if outs else []
    return "\n".join(head + lines + tail) + "\n", local_arrays, written


def translate(source: str) -> CProgram:
    """Parse the C function and lower it (no analysis)."""
    rtype, name, params, body = _parse_function(tokenize(source))
    py, local_arrays, written = _lower(name, params, body)
    return CProgram(source, name, params, local_arrays, written, py, rtype)


def analyse(source: str) -> CProgram:
    """Parse, lower, and run the common analysis and binding."""
    cp = translate(source)
    cp.program = fe.analyse(cp.python)
    return cp


def program_args(cp: CProgram, values: Dict[str, object]) -> Dict[str, object]:
    """The lowered function's arguments: the caller's arrays and scalars, with
    the program's local arrays zero-filled."""
    args = dict(values)
    shape = None
    for q in cp.params:
        if q.dims:
            shape = np.asarray(values[q.name]).shape
            break
    for nm in cp.local_arrays:
        args.setdefault(nm, np.zeros(shape, np.float32))
    return args


def offload(cp: CProgram, values: Dict[str, object], gene: int, **kw):
    """Run the program through the library with a loop gene (see frontend.offload)."""
    return fe.offload(cp.program, program_args(cp, values), gene, **kw)


def run_c(cp: CProgram, values: Dict[str, object], workdir: Optional[str] = None):
    """Compile the original C program with gcc and run it on the given numpy
    arrays (FP32, updated in place) and scalars; returns its return value
    (None for a void function). Every array must have the shape its declared
    dimensions give. The call runs on a thread with a stack large enough for
    the program's local arrays."""
    shape = next(np.asarray(values[q.name]).shape for q in cp.params if q.dims)
    dim_vals: Dict[str, int] = {}
    for q in cp.params:
        if q.dims:
            for dname, n in zip(q.dims, shape):
                dim_vals[dname] = n
            break
    argtypes, args = [], []
    for q in cp.params:
        if q.dims:
            a = values[q.name]
            if not (isinstance(a, np.ndarray) and a.dtype == np.float32 and a.flags.c_contiguous):
                raise FrontendError(f"C: {q.name} must be a C-contiguous float32 array")
            want = tuple(dim_vals.get(d) for d in q.dims)
            if None in want or a.shape != want:
                raise FrontendError(f"C: {q.name} has shape {a.shape}, its declaration asks for {q.dims}")
            argtypes.append(ctypes.c_void_p)
            args.append(a.ctypes.data)
        elif q.name in dim_vals:
            argtypes.append(ctypes.c_int)
            args.append(int(dim_vals[q.name]))
        elif q.ctype == "int":
            argtypes.append(ctypes.c_int)
            args.append(int(values[q.name]))
        else:
            argtypes.append(ctypes.c_float if q.ctype == "float" else ctypes.c_double)
            args.append(float(values[q.name]))
    local_bytes = sum(4 * int(np.prod([dim_vals.get(d, 0) for d in dims])) for dims in cp.local_arrays.values())

    with tempfile.TemporaryDirectory(prefix="ofl_c_", dir=workdir) as d:
        src = os.path.join(d, "program.c")
        lib = os.path.join(d, "libprogram.so")
        with open(src, "w") as f:
            f.write(cp.source)
        r = subprocess.run(["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-o", lib, src], capture_output=True,
                           text=True)
        if r.returncode != 0:
            raise FrontendError(f"C: gcc failed: {r.stderr.strip()[:2000]}")
        so = ctypes.CDLL(lib)
    fn = getattr(so, cp.func)
    fn.argtypes = argtypes
    fn.restype = {"float": ctypes.c_float, "double": ctypes.c_double, "int": ctypes.c_int, "void": None}[cp.rtype]

    out: Dict[str, object] = {}

    def call():
        try:
            out["ret"] = fn(*args)
        except BaseException as e:  # handed back to the caller's thread
            out["error"] = e

    old = threading.stack_size()
    threading.stack_size(max(64 << 20, 2 * local_bytes + (16 << 20)))
    try:
        t = threading.Thread(target=call)
        t.start()
    finally:
        threading.stack_size(old)
    t.join()
    if "error" in out:
        raise out["error"]
    return out["ret"]
