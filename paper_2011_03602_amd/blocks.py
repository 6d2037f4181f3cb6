"""Function-block offload for Python programs (Sec. 3.2.2, Sec. 4.2.1).

The code is analysed for the library routines it calls. Each call is looked up
by the called library's name in a code-pattern table. The table stands in for
the paper's pattern database, and name matching is the lookup the paper
describes; similarity detection of copied code is not done here. A call found
there becomes a function block, which can run on the host as written or be
replaced by the library's GPU routine. The replacement is an ``ast``
rewrite: the call becomes a call of a dispatcher that runs either the
original routine or the GPU one, per block.

Trials follow Sec. 4.2.1. Each block is measured offloaded and not, on its
own. Every combination of the blocks that sped up on their own is then
measured, and the fastest pattern whose results match the original program
wins. A pattern whose results differ gets infinite time. A block whose
operands the GPU routine cannot take (not 2-D floating-point matrices) cannot
be built and scores nothing.

The GPU routine for matrix products is ``ofl_gemm_f32``, the library's FP32
MFMA kernel. Operands move to the device and the product comes back inside
the block: the block's interface to the rest of the program stays a host
array.
"""

from __future__ import annotations

import ast
import itertools
import time
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

from . import ofl_gemm_f32
from .frontend import FrontendError

# called library name -> the GPU routine that replaces it
PATTERNS: Dict[str, str] = {
    "numpy.matmul": "gemm_f32",
    "numpy.dot": "gemm_f32",
    "operator @": "gemm_f32",
}

HOST_ROUTINES: Dict[str, Callable] = {
    "numpy.matmul": np.matmul,
    "numpy.dot": np.dot,
    "operator @": lambda a, b: a @ b,
}


@dataclass
class Block:
    index: int          # source order
    name: str           # the called library name, as matched
    routine: str        # the GPU routine from the pattern table
    line: int
    text: str           # the call as written


@dataclass
class BlockProgram:
    source: str
    func: str
    blocks: List[Block]
    code: object = field(repr=False)   # the module with every block call routed through the dispatcher


def _aliases(tree: ast.Module) -> Dict[str, str]:
    """Local name -> module name, from the source's import statements."""
    out = {}
    for node in ast.walk(tree):
        if isinstance(node, ast.Import):
            for a in node.names:
                out[a.asname or a.name] = a.name
        elif isinstance(node, ast.ImportFrom) and node.module:
            for a in node.names:
                out[a.asname or a.name] = f"{node.module}.{a.name}"
    return out


def _called_name(call: ast.Call, aliases: Dict[str, str]) -> Optional[str]:
    f = call.func
    if isinstance(f, ast.Attribute) and isinstance(f.value, ast.Name):
        mod = aliases.get(f.value.id)
        return f"{mod}.{f.attr}" if mod else None
    if isinstance(f, ast.Name):
        return aliases.get(f.id)
    return None


def analyse_blocks(source: str) -> BlockProgram:
    """Find the calls of library routines the pattern table knows."""
    tree = ast.parse(source)
    funcs = [n for n in tree.body if isinstance(n, ast.FunctionDef)]
    if len(funcs) != 1:
        raise FrontendError("the source must define exactly one function")
    aliases = _aliases(tree)
    found = []
    for node in ast.walk(funcs[0]):
        name = None
        if isinstance(node, ast.Call):
            name = _called_name(node, aliases)
            if name in PATTERNS and (len(node.args) != 2 or node.keywords):
                raise FrontendError(f"line {node.lineno}: {name} with other than two positional operands")
        elif isinstance(node, ast.BinOp) and isinstance(node.op, ast.MatMult):
            name = "operator @"
        if name in PATTERNS:
            found.append((node.lineno, node.col_offset, name, node))
    found.sort(key=lambda x: (x[0], x[1]))
    blocks = []
    for t, (line, _, name, node) in enumerate(found):
        node._ofl_block = t  # marks the node for the rewrite
        blocks.append(Block(t, name, PATTERNS[name], line, ast.unparse(node)))
    tree = ast.fix_missing_locations(_Rewrite().visit(tree))
    return BlockProgram(source, funcs[0].name, blocks, compile(tree, "<program>", "exec"))


class _Rewrite(ast.NodeTransformer):
    def visit_Call(self, node):
        self.generic_visit(node)
        if hasattr(node, "_ofl_block"):
            return ast.copy_location(ast.Call(ast.Name("__ofl_block", ast.Load()),
                                              [ast.Constant(node._ofl_block), *node.args], []), node)
        return node

    def visit_BinOp(self, node):
        self.generic_visit(node)
        if hasattr(node, "_ofl_block"):
            return ast.copy_location(ast.Call(ast.Name("__ofl_block", ast.Load()),
                                              [ast.Constant(node._ofl_block), node.left, node.right], []), node)
        return node


class BlockNotBuildable(FrontendError):
    """The operands of an offloaded block do not fit its GPU routine."""


def gemm_on_gpu(a, b) -> np.ndarray:
    """The GPU routine of a matrix-product block: operands to the device, the
    library's MFMA kernel, the product back to the host."""
    import torch

    a = np.asarray(a)
    b = np.asarray(b)
    if a.ndim != 2 or b.ndim != 2 or a.shape[1] != b.shape[0]:
        raise BlockNotBuildable(f"operands {a.shape} and {b.shape} are not a 2-D matrix product")
    if not (np.issubdtype(a.dtype, np.floating) and np.issubdtype(b.dtype, np.floating)):
        raise BlockNotBuildable("operands are not floating point")
    M, K = a.shape
    N = b.shape[1]
    da = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()
    db = torch.from_numpy(np.ascontiguousarray(b, dtype=np.float32)).cuda()
    dc = torch.empty((M, N), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()
    ofl_gemm_f32(M, N, K, da.data_ptr(), K, db.data_ptr(), N, dc.data_ptr(), N, stream.cuda_stream)
    return dc.cpu().numpy()


GPU_ROUTINES: Dict[str, Callable] = {"gemm_f32": gemm_on_gpu}


def compile_blocks(prog: BlockProgram, gene: int, gpu_routines: Optional[Dict[str, Callable]] = None,
                   host_routines: Optional[Dict[str, Callable]] = None) -> Callable:
    """The program with block b on the GPU where bit b of gene is 1 (the
    routine tables can be replaced, e.g. to test the trials without a GPU)."""
    routines = gpu_routines or GPU_ROUTINES
    hosts = host_routines or HOST_ROUTINES
    blocks = prog.blocks

    def dispatch(t, a, b):
        blk = blocks[t]
        if (gene >> t) & 1:
            return routines[blk.routine](a, b)
        return hosts[blk.name](a, b)

    ns: Dict[str, object] = {"__ofl_block": dispatch}
    exec(prog.code, ns)  # noqa: S102 - the caller's own program
    return ns[prog.func]


@dataclass
class Trial:
    gene: int
    seconds: float          # median of the timed runs; inf when wrong or not buildable
    status: str             # "ok", "wrong" or "not buildable"
    max_rel_err: float = 0.0


def _max_rel(out, ref) -> float:
    outs = out if isinstance(out, tuple) else (out,)
    refs = ref if isinstance(ref, tuple) else (ref,)
    worst = 0.0
    for o, r in zip(outs, refs):
        if o is None or r is None:
            if o is not r:
                return float("inf")
            continue
        o = np.asarray(o, dtype=np.float64)
        r = np.asarray(r, dtype=np.float64)
        if o.shape != r.shape:
            return float("inf")
        if r.size == 0:
            continue
        scale = max(float(np.max(np.abs(r))), 1e-300)
        worst = max(worst, float(np.max(np.abs(o - r))) / scale)
    return worst


def trial_blocks(prog: BlockProgram, args: Dict[str, object], repeats: int = 3, tolerance: float = 1e-4,
                 gpu_routines: Optional[Dict[str, Callable]] = None,
                 host_routines: Optional[Dict[str, Callable]] = None) -> Dict[str, object]:
    """Sec. 4.2.1 trials: every block alone, then every combination of the
    blocks that sped up alone; returns the trials and the best gene. Each
    pattern's result is compared with the original program's (all blocks on
    the host) at the given relative tolerance."""
    n = len(prog.blocks)

    def measure(gene) -> Trial:
        fn = compile_blocks(prog, gene, gpu_routines, host_routines)
        times, out = [], None
        try:
            for _ in range(repeats):
                t0 = time.perf_counter()
                out = fn(**args)
                times.append(time.perf_counter() - t0)
        except BlockNotBuildable:
            return Trial(gene, float("inf"), "not buildable")
        times.sort()
        err = _max_rel(out, reference) if gene else 0.0
        if err > tolerance:
            return Trial(gene, float("inf"), "wrong", err)
        return Trial(gene, times[len(times) // 2], "ok", err)

    reference = compile_blocks(prog, 0, gpu_routines, host_routines)(**args)
    trials = {0: measure(0)}
    for b in range(n):
        trials[1 << b] = measure(1 << b)
    faster = [b for b in range(n) if trials[1 << b].seconds < trials[0].seconds]
    for r in range(2, len(faster) + 1):
        for combo in itertools.combinations(faster, r):
            gene = sum(1 << b for b in combo)
            trials[gene] = measure(gene)
    best = min(trials.values(), key=lambda t: t.seconds)
    return {"trials": [trials[g] for g in sorted(trials)], "best": best, "faster_alone": faster}
