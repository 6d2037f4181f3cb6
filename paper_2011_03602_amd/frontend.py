"""Python programs on the same boundary: a second source language.

The paper's loop offload is language-independent. Code analysis, loop and
variable identification, the gene, the transfer rules and the measured search
are common, and only the parsing is per language (Sec. 3.2.1, Sec. 4.3). This
module is the Python front end. It reads the source of a Python function
written with plain ``for`` loops over ``range()`` and subscripted arrays, and
derives from it what the C library holds as its own program table:

- the loop statements in program order, and the offload screen of Sec. 4.2.2:
  a loop can open a GPU region when its trips are independent. That means
  every array it writes is accessed only at the trip's own index along the
  loop variable, and every scalar it assigns is private to a trip or is a sum
  reduction;
- the iteration loop (the outer loop that fails the screen) and the nests in
  it, each with the arrays it reads, the arrays it writes, and the arrays it
  writes only in part while the rest stays live. The last set comes from the
  index ranges of the accesses;
- the arrays the program references after the loop.

The nests are matched to the library's nests by what they compute. Each
nest's assignment is expanded into a polynomial in the loaded array values
and the scalars. The program's arrays are bound to the library's by their
place in those polynomials: which neighbour of p each one multiplies, and with
which sign. Their names play no part. A program that does not compute the
library's nests is rejected with FrontendError, because no kernel exists for
it.

The plans and the runs go through the same C interface. ``Program.plan``
hands the analysed variable sets to ofl_plan_nests. ``offload`` and
``search`` run the bound arrays through ofl_set_loop_gene, ofl_jacobi_run and
ofl_grid_search_loops.
"""

from __future__ import annotations

import ast
import time
from dataclasses import dataclass, field
from fractions import Fraction
from typing import Dict, List, Optional, Tuple

import numpy as np

from . import (ARRAY_NAMES, OFL_XFER_HOISTED, Grid, ofl_get_stats, ofl_grid_search_loops, ofl_jacobi_run,
               ofl_plan_nests, ofl_program_vars, ofl_set_loop_gene)

NEST_NAMES = ("S", "R", "C")


class FrontendError(ValueError):
    """The program uses a construct the front end does not read, or computes
    something the library has no kernel for."""


# ------------------------------------------------------------ linear forms


@dataclass(frozen=True)
class Lin:
    """An integer linear form: sum of coef*symbol plus a constant."""

    terms: Tuple[Tuple[str, int], ...] = ()
    const: int = 0

    @staticmethod
    def of(sym: Optional[str] = None, const: int = 0) -> "Lin":
        return Lin(((sym, 1),) if sym else (), const)

    def _dict(self):
        return dict(self.terms)

    def __add__(self, o: "Lin") -> "Lin":
        d = self._dict()
        for s, c in o.terms:
            d[s] = d.get(s, 0) + c
        return Lin(tuple(sorted((s, c) for s, c in d.items() if c)), self.const + o.const)

    def __neg__(self) -> "Lin":
        return Lin(tuple((s, -c) for s, c in self.terms), -self.const)

    def __sub__(self, o: "Lin") -> "Lin":
        return self + (-o)

    def scale(self, k: int) -> "Lin":
        return Lin(tuple((s, c * k) for s, c in self.terms if c * k), self.const * k)

    def var_offset(self) -> Tuple[Optional[str], Optional[int]]:
        """(symbol, offset) when the form is symbol + constant, else (None, None)."""
        if len(self.terms) == 1 and self.terms[0][1] == 1:
            return self.terms[0][0], self.const
        return None, None

    def minus(self, o: "Lin") -> Optional[int]:
        """self - o as an integer when the symbols cancel, else None."""
        d = self - o
        return d.const if not d.terms else None

    def evaluate(self, env: Dict[str, int]) -> int:
        return self.const + sum(c * int(env[s]) for s, c in self.terms)


def lin(node: ast.AST) -> Lin:
    if isinstance(node, ast.Constant) and isinstance(node.value, int) and not isinstance(node.value, bool):
        return Lin.of(None, node.value)
    if isinstance(node, ast.Name):
        return Lin.of(node.id)
    if isinstance(node, ast.UnaryOp) and isinstance(node.op, ast.USub):
        return -lin(node.operand)
    if isinstance(node, ast.BinOp) and isinstance(node.op, (ast.Add, ast.Sub)):
        a, b = lin(node.left), lin(node.right)
        return a + b if isinstance(node.op, ast.Add) else a - b
    if isinstance(node, ast.BinOp) and isinstance(node.op, ast.Mult):
        a, b = lin(node.left), lin(node.right)
        if not a.terms:
            return b.scale(a.const)
        if not b.terms:
            return a.scale(b.const)
    raise FrontendError(f"line {getattr(node, 'lineno', '?')}: not an integer linear form: {ast.unparse(node)}")


# ----------------------------------------------------------------- program


@dataclass
class Access:
    array: str
    index: Tuple[Lin, ...]
    store: bool


@dataclass
class Loop:
    index: int              # program order
    var: str
    lo: Lin
    hi: Lin                 # range(lo, hi)
    depth: int              # 0 for a loop directly in the function body
    parent: Optional[int]
    node: ast.For
    parallel: bool = False
    reason: str = ""        # why the screen refused it


@dataclass
class Nest:
    name: str                       # S, R or C (after binding)
    loops: List[int]                # its k, j, i loops (program order)
    reads: List[str]
    writes: List[str]
    partial: List[str]
    reduction: Optional[str] = None


@dataclass
class Program:
    """What the front end read from one Python function."""

    source: str
    func: str
    params: List[str]
    shape_syms: Tuple[str, ...]
    loops: List[Loop]
    iter_loop: int
    nests: List[Nest]
    arrays: List[str]               # every array of the program, in first-use order
    live_after: List[str]
    returns: List[str]
    binding: Dict[str, str] = field(default_factory=dict)   # program array -> library array name
    symbols: Dict[str, str] = field(default_factory=dict)   # library scalar -> program scalar

    def loop_table(self) -> List[Tuple[int, int, int]]:
        """(nest, level, parallel) per loop in program order; nest -1 for the iteration loop
        (the same layout as ofl_loop_table, extents aside)."""
        out = []
        for lp in self.loops:
            nest = next((n for n, x in enumerate(self.nests) if lp.index in x.loops), -1)
            level = self.nests[nest].loops.index(lp.index) if nest >= 0 else -1
            out.append((nest, level, int(lp.parallel)))
        return out

    def nest_vars(self, ids: Dict[str, int]) -> List[Tuple[int, int, int]]:
        """(reads, writes, partial) bit sets per nest under the array numbering ids."""
        bits = lambda names: sum(1 << ids[a] for a in set(names))  # noqa: E731
        return [(bits(n.reads), bits(n.writes), bits(n.partial)) for n in self.nests]

    def plan(self, mask: int, xfer_mode: int, iters: int, sync_host_at_end: bool = True):
        """The transfers of a gene, from the analysed variable sets, by the library's planner.
        Arrays are numbered in first-use order; returns (transfers, array names)."""
        ids = {a: t for t, a in enumerate(self.arrays)}
        live = sum(1 << ids[a] for a in self.live_after)
        xs, _, _ = ofl_plan_nests(self.nest_vars(ids), len(self.arrays), live, mask, xfer_mode, iters,
                                  sync_host_at_end)
        return xs, list(self.arrays)


def _subscript(node: ast.Subscript) -> Tuple[str, Tuple[Lin, ...]]:
    if not isinstance(node.value, ast.Name):
        raise FrontendError(f"line {node.lineno}: subscripts must index a named array")
    sl = node.slice
    elts = sl.elts if isinstance(sl, ast.Tuple) else [sl]
    return node.value.id, tuple(lin(e) for e in elts)


class _Collector(ast.NodeVisitor):
    """Array accesses and scalar uses of a statement list, in execution order."""

    def __init__(self):
        self.accesses: List[Access] = []
        self.scalar_events: List[Tuple[str, str]] = []   # (name, 'load' | 'store' | 'sum')

    def load_expr(self, node):
        for sub in ast.walk(node):
            if isinstance(sub, ast.Subscript):
                a, idx = _subscript(sub)
                self.accesses.append(Access(a, idx, False))
            elif isinstance(sub, ast.Name) and isinstance(sub.ctx, ast.Load):
                self.scalar_events.append((sub.id, "load"))

    def stmts(self, body):
        for st in body:
            if isinstance(st, ast.Assign):
                self.load_expr(st.value)
                for t in st.targets:
                    self.target(t)
            elif isinstance(st, ast.AugAssign):
                if isinstance(st.target, ast.Name):
                    self.load_expr(st.value)
                    kind = "sum" if isinstance(st.op, ast.Add) else "store"
                    if kind == "store":
                        self.scalar_events.append((st.target.id, "load"))
                    self.scalar_events.append((st.target.id, kind))
                else:
                    self.load_expr(st.value)
                    a, idx = _subscript(st.target)
                    self.accesses.append(Access(a, idx, False))
                    self.accesses.append(Access(a, idx, True))
            elif isinstance(st, ast.For):
                self.stmts(st.body)
            elif isinstance(st, (ast.Expr, ast.Pass)):
                if isinstance(st, ast.Expr):
                    self.load_expr(st.value)
            else:
                raise FrontendError(f"line {st.lineno}: statement not read by the front end: "
                                    f"{type(st).__name__}")

    def target(self, t):
        if isinstance(t, ast.Subscript):
            self.load_expr(t.slice)
            a, idx = _subscript(t)
            self.accesses.append(Access(a, idx, True))
        elif isinstance(t, ast.Name):
            self.scalar_events.append((t.id, "store"))
        elif isinstance(t, ast.Tuple):
            for e in t.elts:
                self.target(e)
        else:
            raise FrontendError(f"line {t.lineno}: assignment target not read by the front end")


def _collect(body) -> _Collector:
    c = _Collector()
    c.stmts(body)
    return c


def _screen(loop: Loop, loop_vars: set) -> Tuple[bool, str]:
    """Sec. 4.2.2 screen: can the trips of this loop run in parallel?"""
    c = _collect(loop.node.body)
    v = loop.var
    own = Lin.of(v)
    for a in sorted({x.array for x in c.accesses if x.store}):
        acc = [x for x in c.accesses if x.array == a]
        dims = set(range(len(acc[0].index)))
        for x in acc:
            dims &= {d for d, e in enumerate(x.index) if e == own}
        if not dims:
            return False, f"{a} is written and accessed across trips of {v}"
    seen = {}
    for name, kind in c.scalar_events:
        if name in loop_vars:
            continue
        seen.setdefault(name, []).append(kind)
    for name, kinds in seen.items():
        if "store" not in kinds and "sum" not in kinds:
            continue  # only read: invariant
        if all(k == "sum" for k in kinds):
            continue  # a sum reduction
        if kinds[0] == "store":
            continue  # assigned before use in every trip: private
        return False, f"scalar {name} is carried across trips of {v}"
    return True, ""


def _poly_const(c) -> Dict:
    return {(): Fraction(c)} if c else {}


def _poly_add(a, b, sign=1):
    out = dict(a)
    for m, c in b.items():
        out[m] = out.get(m, 0) + sign * c
        if out[m] == 0:
            del out[m]
    return out


def _mono_mul(m1, m2):
    d = dict(m1)
    for f, pw in m2:
        d[f] = d.get(f, 0) + pw
        if d[f] == 0:
            del d[f]
    return tuple(sorted(d.items()))


def _poly_mul(a, b):
    out = {}
    for m1, c1 in a.items():
        for m2, c2 in b.items():
            m = _mono_mul(m1, m2)
            out[m] = out.get(m, 0) + c1 * c2
            if out[m] == 0:
                del out[m]
    return out


def _poly(node, env, loop_vars) -> Dict:
    """Expand an expression into {monomial: coefficient}; factors are
    ('a', array, offsets) for array loads and ('s', name) for scalars."""
    if isinstance(node, ast.Constant) and isinstance(node.value, (int, float)):
        return _poly_const(Fraction(node.value))
    if isinstance(node, ast.Name):
        if node.id in env:
            return env[node.id]
        return {((("s", node.id), 1),): Fraction(1)}
    if isinstance(node, ast.Subscript):
        a, idx = _subscript(node)
        offs = []
        for d, e in enumerate(idx):
            var, off = e.var_offset()
            if var != loop_vars[d]:
                raise FrontendError(f"line {node.lineno}: index {d} of {a} is not {loop_vars[d]} + constant")
            offs.append(off)
        return {((("a", a, tuple(offs)), 1),): Fraction(1)}
    if isinstance(node, ast.UnaryOp) and isinstance(node.op, ast.USub):
        return {m: -c for m, c in _poly(node.operand, env, loop_vars).items()}
    if isinstance(node, ast.BinOp):
        a = _poly(node.left, env, loop_vars)
        if isinstance(node.op, ast.Pow):
            if not (isinstance(node.right, ast.Constant) and isinstance(node.right.value, int)
                    and node.right.value >= 0):
                raise FrontendError(f"line {node.lineno}: only non-negative integer powers")
            out = _poly_const(1)
            for _ in range(node.right.value):
                out = _poly_mul(out, a)
            return out
        b = _poly(node.right, env, loop_vars)
        if isinstance(node.op, ast.Add):
            return _poly_add(a, b)
        if isinstance(node.op, ast.Sub):
            return _poly_add(a, b, -1)
        if isinstance(node.op, ast.Mult):
            return _poly_mul(a, b)
        if isinstance(node.op, ast.Div):
            if len(b) != 1:
                raise FrontendError(f"line {node.lineno}: division by a sum")
            (m, c), = b.items()
            inv = {tuple((f, -pw) for f, pw in m): 1 / c}
            return _poly_mul(a, inv)
    raise FrontendError(f"line {getattr(node, 'lineno', '?')}: expression not read by the front end: "
                        f"{ast.unparse(node)}")


def _nest_polys(loop_node: ast.For, loop_vars) -> Tuple[Optional[Tuple[str, tuple]], Dict, Optional[str]]:
    """Expand the innermost body of a perfect nest: (store target (array, offsets)
    or None, polynomial of the stored / summed value, reduction scalar or None)."""
    env: Dict[str, Dict] = {}
    target, poly, red = None, None, None
    for st in loop_node.body:
        if isinstance(st, ast.Assign) and len(st.targets) == 1 and isinstance(st.targets[0], ast.Name):
            env[st.targets[0].id] = _poly(st.value, env, loop_vars)
        elif isinstance(st, ast.Assign) and len(st.targets) == 1 and isinstance(st.targets[0], ast.Subscript):
            if target is not None or red is not None:
                raise FrontendError(f"line {st.lineno}: a nest may store one array")
            t = _poly(st.targets[0], {}, loop_vars)
            (m, _), = t.items()
            target = (m[0][0][1], m[0][0][2])
            poly = _poly(st.value, env, loop_vars)
        elif isinstance(st, ast.AugAssign) and isinstance(st.target, ast.Name) and isinstance(st.op, ast.Add):
            if target is not None or red is not None:
                raise FrontendError(f"line {st.lineno}: a nest may hold one reduction")
            red = st.target.id
            poly = _poly(st.value, env, loop_vars)
        else:
            raise FrontendError(f"line {st.lineno}: statement not read in a nest body")
    if poly is None:
        raise FrontendError(f"line {loop_node.lineno}: nest stores nothing")
    return target, poly, red


def _parse(source: str) -> Tuple[ast.FunctionDef, List[Loop]]:
    tree = ast.parse(source)
    funcs = [n for n in tree.body if isinstance(n, ast.FunctionDef)]
    if len(funcs) != 1:
        raise FrontendError("the source must define exactly one function")
    fn = funcs[0]
    loops: List[Loop] = []

    def visit(body, depth, parent):
        for st in body:
            if isinstance(st, ast.For):
                if not isinstance(st.target, ast.Name):
                    raise FrontendError(f"line {st.lineno}: loop target must be a name")
                it = st.iter
                if not (isinstance(it, ast.Call) and isinstance(it.func, ast.Name) and it.func.id == "range"
                        and 1 <= len(it.args) <= 2 and not it.keywords):
                    raise FrontendError(f"line {st.lineno}: loops must run over range(hi) or range(lo, hi)")
                lo, hi = (Lin(), lin(it.args[0])) if len(it.args) == 1 else (lin(it.args[0]), lin(it.args[1]))
                lp = Loop(len(loops), st.target.id, lo, hi, depth, parent, st)
                loops.append(lp)
                visit(st.body, depth + 1, lp.index)
            elif st.__class__.__name__ in ("If", "While", "With", "Try"):
                raise FrontendError(f"line {st.lineno}: {type(st).__name__} is not read by the front end")

    visit(fn.body, 0, None)
    return fn, loops


def screen(source: str) -> List[Tuple[str, int, bool, str]]:
    """The offload screen alone, for any function the front end reads:
    (loop variable, depth, parallel, reason) per loop in program order."""
    _, loops = _parse(source)
    loop_vars = {lp.var for lp in loops}
    out = []
    for lp in loops:
        ok, why = _screen(lp, loop_vars)
        out.append((lp.var, lp.depth, ok, why))
    return out


def _range_along(index: Lin, loops_by_var: Dict[str, Loop]) -> Optional[Tuple[Lin, Lin]]:
    var, off = index.var_offset()
    if var is None or var not in loops_by_var:
        return None
    lp = loops_by_var[var]
    return lp.lo + Lin.of(None, off), lp.hi + Lin.of(None, off - 1)


def _inside(inner: Tuple[Lin, Lin], outer: Tuple[Lin, Lin]) -> bool:
    lo = inner[0].minus(outer[0])
    hi = outer[1].minus(inner[1])
    return lo is not None and hi is not None and lo >= 0 and hi >= 0


def analyse(source: str) -> Program:
    """Read a Python function and bind it to the library's program."""
    fn, loops = _parse(source)
    params = [a.arg for a in fn.args.args]
    shape_syms: Tuple[str, ...] = ()
    for st in fn.body:
        if (isinstance(st, ast.Assign) and isinstance(st.targets[0], ast.Tuple)
                and isinstance(st.value, ast.Attribute) and st.value.attr == "shape"):
            shape_syms = tuple(e.id for e in st.targets[0].elts)
            break
    loop_vars = {lp.var for lp in loops}
    for lp in loops:
        lp.parallel, lp.reason = _screen(lp, loop_vars)
    tops = [lp for lp in loops if lp.depth == 0]
    if len(tops) != 1 or tops[0].parallel:
        raise FrontendError("the function must hold one iteration loop whose trips depend on each other")
    it_loop = tops[0]
    # nests: perfect 3-deep loop nests directly inside the iteration loop
    nests: List[Nest] = []
    for st in it_loop.node.body:
        if isinstance(st, ast.For):
            chain = [st]
            while len(chain[-1].body) == 1 and isinstance(chain[-1].body[0], ast.For):
                chain.append(chain[-1].body[0])
            if len(chain) != 3:
                raise FrontendError(f"line {st.lineno}: nests must be three perfectly nested loops")
            ids = [next(lp.index for lp in loops if lp.node is n) for n in chain]
            c = _collect(chain[-1].body)
            nests.append(Nest("", ids, [x.array for x in c.accesses if not x.store],
                              [x.array for x in c.accesses if x.store], []))
        elif not (isinstance(st, ast.Assign) and len(st.targets) == 1 and isinstance(st.targets[0], ast.Name)):
            raise FrontendError(f"line {st.lineno}: the iteration loop may hold nests and scalar assignments")
    if len(nests) != 3:
        raise FrontendError(f"the iteration loop holds {len(nests)} nests; the library's program has 3")
    for n in nests:
        for lid in n.loops:
            if not loops[lid].parallel:
                raise FrontendError(f"loop over {loops[lid].var} fails the screen: {loops[lid].reason}")
    if not shape_syms:
        raise FrontendError("unpack the array shape first (K, J, I = p.shape)")
    for n in nests:
        for d, lid in enumerate(n.loops):
            lp = loops[lid]
            # the library's nests run over the interior along every axis
            if lp.lo != Lin.of(None, 1) or lp.hi != Lin.of(shape_syms[d], -1):
                raise FrontendError(f"line {lp.node.lineno}: loop over {lp.var} must run over "
                                    f"range(1, {shape_syms[d]} - 1), the interior")
    arrays: List[str] = []
    for x in _collect(it_loop.node.body).accesses:
        if x.array not in arrays:
            arrays.append(x.array)
    # after the loop: what the program references (and returns)
    after = fn.body[fn.body.index(it_loop.node) + 1:]
    live_after, returns = [], []
    for st in after:
        for sub in ast.walk(st):
            if isinstance(sub, ast.Name) and isinstance(sub.ctx, ast.Load) and sub.id in arrays:
                if sub.id not in live_after:
                    live_after.append(sub.id)
        if isinstance(st, ast.Return) and st.value is not None:
            vals = st.value.elts if isinstance(st.value, ast.Tuple) else [st.value]
            for v in vals:
                if not isinstance(v, ast.Name):
                    raise FrontendError(f"line {st.lineno}: return names only")
                returns.append(v.id)
    # partial writes: a nest writes part of an array whose rest stays live
    reads_by_nest = []  # per nest: (read access, that nest's loops by variable)
    for m in nests:
        mvars = {loops[i].var: loops[i] for i in m.loops}
        reads_by_nest.append([(x, mvars) for x in _collect(loops[m.loops[-1]].node.body).accesses if not x.store])
    for n in nests:
        by_var = {loops[i].var: loops[i] for i in n.loops}
        c = _collect(loops[n.loops[-1]].node.body)
        for a in dict.fromkeys(x.array for x in c.accesses if x.store):
            wr = [x for x in c.accesses if x.store and x.array == a][0]
            ndim = len(wr.index)
            if len(shape_syms) != ndim:
                raise FrontendError("unpack the array shape first (K, J, I = p.shape)")
            box = [_range_along(e, by_var) for e in wr.index]
            if any(b is None for b in box):
                raise FrontendError(f"{a} is stored at an index that is not loop variable + constant")
            full = [(Lin(), Lin.of(s, -1)) for s in shape_syms]
            if all(box[d][0] == full[d][0] and box[d][1] == full[d][1] for d in range(ndim)):
                continue
            live = a in live_after  # the caller sees the whole array after the loop
            for x, mvars in (r for rs in reads_by_nest for r in rs):
                if x.array != a or live:
                    continue
                rbox = [_range_along(e, mvars) for e in x.index]
                if any(r is None for r in rbox) or not all(_inside(rbox[d], box[d]) for d in range(ndim)):
                    live = True  # some nest reads it where this nest does not write
            if live:
                n.partial.append(a)
    prog = Program(source, fn.name, params, shape_syms, loops, it_loop.index, nests, arrays, live_after, returns)
    _bind(prog)
    _check_iteration_body(prog)
    return prog


# ----------------------------------------------------------------- binding

# The library's nests written in the same language: the pattern a program's
# nests are matched against (what the kernels compute, as polynomials).
_LIBRARY_SOURCE = '''
def library(p, wrk2, a0, a1, a2, a3, b0, b1, b2, c0, c1, c2, bnd, wrk1, iters, omega):
    K, J, I = p.shape
    for n in range(iters):
        gosa = 0.0
        for k in range(1, K - 1):
            for j in range(1, J - 1):
                for i in range(1, I - 1):
                    s0 = (a0[k, j, i] * p[k, j, i + 1] + a1[k, j, i] * p[k, j + 1, i]
                          + a2[k, j, i] * p[k + 1, j, i]
                          + b0[k, j, i] * (p[k, j + 1, i + 1] - p[k, j - 1, i + 1]
                                           - p[k, j + 1, i - 1] + p[k, j - 1, i - 1])
                          + b1[k, j, i] * (p[k + 1, j + 1, i] - p[k + 1, j - 1, i]
                                           - p[k - 1, j + 1, i] + p[k - 1, j - 1, i])
                          + b2[k, j, i] * (p[k + 1, j, i + 1] - p[k + 1, j, i - 1]
                                           - p[k - 1, j, i + 1] + p[k - 1, j, i - 1])
                          + c0[k, j, i] * p[k, j, i - 1] + c1[k, j, i] * p[k, j - 1, i]
                          + c2[k, j, i] * p[k - 1, j, i] + wrk1[k, j, i])
                    ss = (s0 * a3[k, j, i] - p[k, j, i]) * bnd[k, j, i]
                    wrk2[k, j, i] = p[k, j, i] + omega * ss
        for k in range(1, K - 1):
            for j in range(1, J - 1):
                for i in range(1, I - 1):
                    d = (wrk2[k, j, i] - p[k, j, i]) / omega
                    gosa += d * d
        for k in range(1, K - 1):
            for j in range(1, J - 1):
                for i in range(1, I - 1):
                    p[k, j, i] = wrk2[k, j, i]
    return p, gosa
'''


def _nest_forms(prog_fn_loops, nest: Nest):
    loops = [prog_fn_loops[i] for i in nest.loops]
    return _nest_polys(loops[-1].node, [lp.var for lp in loops])


def _colours(forms: List[Tuple]) -> Dict[Tuple[str, str], tuple]:
    """Colour refinement over the arrays and scalars of the nests' polynomials:
    a name's colour is what it multiplies, at which offsets, with which
    coefficient, in which nest; refined until stable."""
    names = set()
    for _, poly, _ in forms:
        for m in poly:
            for f, _ in m:
                names.add((f[0], f[1]))
    for target, _, red in forms:
        if target:
            names.add(("a", target[0]))
        if red:
            names.add(("s", red))
    col = {x: (x[0],) for x in names}
    for _ in range(8):
        sig = {}
        for x in names:
            items = []
            for t, (target, poly, red) in enumerate(forms):
                if target and ("a", target[0]) == x:
                    items.append(("store", t, target[1]))
                if red and ("s", red) == x:
                    items.append(("sum", t))
                for m, c in poly.items():
                    mine = [(f[2] if f[0] == "a" else None, pw) for f, pw in m if (f[0], f[1]) == x]
                    if not mine:
                        continue
                    rest = sorted((col[(f[0], f[1])], f[2] if f[0] == "a" else None, pw) for f, pw in m)
                    items.append((t, tuple(sorted(mine, key=repr)), str(c), tuple(rest)))
            sig[x] = (col[x], tuple(sorted(items, key=repr)))
        keys = sorted(set(sig.values()), key=repr)
        new = {x: (x[0], keys.index(sig[x])) for x in names}
        if len(set(new.values())) == len(set(col.values())):
            col = new
            break
        col = new
    return {x: (col[x][0], sig[x]) for x in names}


_LIB_CACHE: Dict[str, object] = {}


def _library():
    if "prog" not in _LIB_CACHE:
        fn, loops = _parse(_LIBRARY_SOURCE)
        it = next(lp for lp in loops if lp.depth == 0)
        nests = []
        for st in it.node.body:
            if isinstance(st, ast.For):
                chain = [st, st.body[0], st.body[0].body[0]]
                nests.append(Nest("", [next(lp.index for lp in loops if lp.node is n) for n in chain], [], [], []))
        forms = [_nest_forms(loops, n) for n in nests]
        _LIB_CACHE["prog"] = (forms, _colours(forms))
    return _LIB_CACHE["prog"]


def _bind(prog: Program):
    forms = [_nest_forms(prog.loops, n) for n in prog.nests]
    lib_forms, lib_col = _library()
    col = _colours(forms)
    by_colour: Dict[tuple, List[Tuple[str, str]]] = {}
    for x, c in lib_col.items():
        by_colour.setdefault(c, []).append(x)
    binding: Dict[Tuple[str, str], Tuple[str, str]] = {}
    for x, c in col.items():
        match = by_colour.get(c, [])
        if len(match) != 1:
            raise FrontendError(f"{x[1]}: no single counterpart in the library's nests "
                                "(the program does not compute what the kernels compute)")
        binding[x] = match[0]
    if len(set(binding.values())) != len(binding) or len(binding) != len(lib_col):
        raise FrontendError("the program's variables do not map one to one onto the library's")

    def rename(poly):
        out = {}
        for m, c in poly.items():
            mm = []
            for f, pw in m:
                to = binding[(f[0], f[1])]
                mm.append(((f[0], to[1]) + tuple(f[2:]), pw))
            out[tuple(sorted(mm))] = c
        return out

    for t, ((target, poly, red), (lt, lpoly, lred)) in enumerate(zip(forms, lib_forms)):
        ok = rename(poly) == lpoly
        ok = ok and ((target is None) == (lt is None)) and ((red is None) == (lred is None))
        if target is not None:
            ok = ok and binding[("a", target[0])][1] == lt[0] and target[1] == lt[1]
        if red is not None:
            ok = ok and binding[("s", red)][1] == lred
        if not ok:
            raise FrontendError(f"nest {t + 1} does not compute the library's nest {NEST_NAMES[t]}")
        prog.nests[t].name = NEST_NAMES[t]
        prog.nests[t].reduction = red
    prog.binding = {x[1]: to[1] for x, to in binding.items() if x[0] == "a"}
    prog.symbols = {to[1]: x[1] for x, to in binding.items() if x[0] == "s"}


def _check_iteration_body(prog: Program):
    """The reduction scalar must restart at zero in every trip of the iteration
    loop (the library returns the residual of the last sweep)."""
    red = prog.symbols.get("gosa")
    it = prog.loops[prog.iter_loop].node
    starts = [st for st in it.body if isinstance(st, ast.Assign) and isinstance(st.targets[0], ast.Name)
              and st.targets[0].id == red]
    if len(starts) != 1 or not (isinstance(starts[0].value, ast.Constant) and starts[0].value.value == 0):
        raise FrontendError(f"{red} must be set to 0 once at the top of every iteration")
    if it.body.index(starts[0]) > next(t for t, st in enumerate(it.body) if isinstance(st, ast.For)):
        raise FrontendError(f"{red} must be set to 0 before the nests")


# --------------------------------------------------------------------- runs


def library_ids(prog: Program) -> Dict[str, int]:
    """Program array -> OFL_ARR_* id."""
    return {a: ARRAY_NAMES.index(lib) for a, lib in prog.binding.items()}


def _grid(prog: Program, args: Dict[str, object], **grid_kw) -> Tuple[Grid, int, np.float32]:
    missing = [a for a in prog.binding if a not in args]
    if missing:
        raise FrontendError(f"arguments missing: {missing}")
    arrays = {lib: np.asarray(args[a]) for a, lib in prog.binding.items()}
    env = {k: v for k, v in args.items() if np.isscalar(v)}
    p_name = next(a for a, lib in prog.binding.items() if lib == "p")
    for d, s in enumerate(prog.shape_syms):
        env[s] = np.asarray(args[p_name]).shape[d]
    it = prog.loops[prog.iter_loop]
    iters = it.hi.evaluate(env) - it.lo.evaluate(env)
    omega = np.float32(args[prog.symbols["omega"]])
    return Grid(arrays, **grid_kw), iters, omega


def _finish(prog: Program, args, g: Grid, gosa: float):
    for a, lib in prog.binding.items():
        if a in prog.live_after:
            np.asarray(args[a])[...] = g.host[lib]
    red = prog.symbols.get("gosa")
    out = [gosa if r == red else args[r] for r in prog.returns]
    return out[0] if len(out) == 1 else tuple(out)


def offload(prog: Program, args: Dict[str, object], gene: int, xfer_mode: int = OFL_XFER_HOISTED,
            stats: Optional[list] = None, timings: Optional[dict] = None, **grid_kw):
    """Run the program with the loop gene (bit b: the b-th loop that passes the
    screen, in program order) through the library. Arrays the program
    references after the loop are written back in place; returns what the
    program returns. timings, if given, receives the seconds spent setting up
    the grid, in ofl_jacobi_run (transfers included) and writing back."""
    t0 = time.perf_counter()
    g, iters, omega = _grid(prog, args, **grid_kw)
    try:
        ofl_set_loop_gene(g.handle, gene, xfer_mode)
        t1 = time.perf_counter()
        gosa = ofl_jacobi_run(g.handle, iters, omega)
        t2 = time.perf_counter()
        if stats is not None:
            stats.append(ofl_get_stats(g.handle))
        out = _finish(prog, args, g, gosa)
        if timings is not None:
            timings.update(setup=t1 - t0, run=t2 - t1, writeback=time.perf_counter() - t2)
        return out
    finally:
        g.close()


def search(prog: Program, args: Dict[str, object], xfer_mode: int = OFL_XFER_HOISTED, ga=None,
           time_limit_ms: float = 0.0, probe_iters: Optional[int] = None, **grid_kw):
    """The loop-gene GA on the program's own data (Sec. 4.2.2); returns the
    search result (its gene is in the program's loop order)."""
    g, iters, omega = _grid(prog, args, **grid_kw)
    try:
        return ofl_grid_search_loops(g.handle, probe_iters or iters, omega, xfer_mode, time_limit_ms, ga)
    finally:
        g.close()


def run_python(source: str, args: Dict[str, object]):
    """Run the program itself, interpreted (small grids only): the original
    program the offloaded runs are checked against."""
    ns: Dict[str, object] = {}
    exec(compile(source, "<program>", "exec"), ns)  # noqa: S102 - the caller's own program
    fn = next(v for k, v in ns.items() if callable(v) and not k.startswith("__"))
    return fn(**args)


def check_against_library(prog: Program) -> None:
    """The analysed loop table and variable sets against the library's own."""
    ids = library_ids(prog)
    lib_vars, lib_live = ofl_program_vars()
    mine = prog.nest_vars(ids)
    if [tuple(x) for x in mine] != [tuple(x) for x in lib_vars]:
        raise FrontendError(f"variable sets differ from the library's: {mine} vs {lib_vars}")
    live = sum(1 << ids[a] for a in prog.live_after)
    if live != lib_live:
        raise FrontendError("the arrays referenced after the loop differ from the library's")
    table = prog.loop_table()
    want = [(-1, -1, 0)] + [(n, lev, 1) for n in range(3) for lev in range(3)]
    if table != want:
        raise FrontendError(f"loop table differs from the library's: {table}")
