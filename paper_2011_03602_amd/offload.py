"""Offload a Python program in the paper's order (Sec. 4.2): function blocks
first, since a block replaced by a tuned GPU routine gains more than its
loops offloaded one by one, then loop offload; the best measured pattern of
each is the solution.

A program whose loops do not form the library's program (no iteration loop
over the three nests, or nests that compute something else) gets no loop
offload, and the report says why. A program without calls of known library
routines has no function blocks.
"""

from __future__ import annotations

from typing import Callable, Dict, Optional

from . import OFL_XFER_HOISTED
from . import blocks as fb
from . import frontend as fe


def offload_program(source: str, args: Dict[str, object], xfer_mode: int = OFL_XFER_HOISTED, ga=None,
                    block_repeats: int = 3, tolerance: float = 1e-4, search_loops: bool = True,
                    gpu_routines: Optional[Dict[str, Callable]] = None) -> Dict[str, object]:
    """Returns {"blocks": ..., "loops": ...}: for the function blocks, the
    trials and the best block gene (None when there are no blocks); for the
    loops, the analysis and, with search_loops, the loop-gene GA's result on
    the program's data (or why the loops cannot be offloaded)."""
    report: Dict[str, object] = {"blocks": None, "loops": None}
    bprog = fb.analyse_blocks(source)
    if bprog.blocks:
        res = fb.trial_blocks(bprog, args, repeats=block_repeats, tolerance=tolerance, gpu_routines=gpu_routines)
        report["blocks"] = {
            "found": [f"{b.name} (line {b.line})" for b in bprog.blocks],
            "trials": [(t.gene, t.seconds, t.status) for t in res["trials"]],
            "best_gene": res["best"].gene,
            "faster_alone": res["faster_alone"],
        }
    try:
        lprog = fe.analyse(source)
    except fe.FrontendError as e:
        report["loops"] = {"offloadable": False, "reason": str(e)}
        return report
    loops = {"offloadable": True, "gene_bits": sum(lp.parallel for lp in lprog.loops),
             "binding": dict(lprog.binding)}
    if search_loops:
        r = fe.search(lprog, args, xfer_mode, ga)
        loops.update(gene=r.gene, mask=r.mask, levels=list(r.level), best_ms=r.best_ms, cpu_ms=r.cpu_ms)
    report["loops"] = loops
    return report
