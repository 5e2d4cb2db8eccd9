"""Checkpoint and restart of a hierarchy run.

The state of a sub-cycled run at a synchronised time is the ghosted state U
of every level (the driver's other buffers, S0, S1, acc and the stage
derivatives k, are overwritten before they are read in every coarse step)
plus the time.  A checkpoint file holds, in safetensors format, one FP64
tensor per level in the library's packed level layout, and as metadata the
hierarchy (N0, xlo, dx0, levels, open), the system parameters, the time, the
step count and any caller entries (JSON).  Restoring builds a new patchset
from the metadata and copies the tensors into fresh device states, so a run
continued from a checkpoint reproduces the uninterrupted run bit for bit.
"""
from __future__ import annotations

import dataclasses
import json

from . import molamr as M

FORMAT = "molamr-checkpoint-1"


def _hier_meta(h: M.Hierarchy) -> dict:
    return {"N0": list(h.N0), "xlo": list(h.xlo), "dx0": h.dx0, "open": bool(h.open),
            "levels": [[int(r), [[list(lo), list(hi)] for lo, hi in boxes]] for r, boxes in h.levels]}


def _hier_from(m: dict) -> M.Hierarchy:
    levels = [(r, [(tuple(lo), tuple(hi)) for lo, hi in boxes]) for r, boxes in m["levels"]]
    return M.Hierarchy(tuple(m["N0"]), tuple(m["xlo"]), m["dx0"], levels, open=m["open"])


def save(path, ps: M.Patchset, states, t: float = 0.0, step: int = 0, extra: dict | None = None) -> None:
    """Write the level states of `ps` (states: list of dicts with "U", as
    alloc_states returns, or a list of U tensors) to `path`."""
    from safetensors.torch import save_file
    Us = [s["U"] if isinstance(s, dict) else s for s in states]
    if len(Us) != ps.nlev:
        raise ValueError(f"{len(Us)} level states for a hierarchy of {ps.nlev} levels")
    tensors = {}
    for l, U in enumerate(Us):
        if U.numel() != ps.layouts[l]["nelems"] or str(U.dtype) != "torch.float64":
            raise ValueError(f"level {l}: expected {ps.layouts[l]['nelems']} float64 values")
        tensors[f"U{l}"] = U.detach().to("cpu").contiguous()
    meta = {"format": FORMAT, "hierarchy": json.dumps(_hier_meta(ps.hier)),
            "system": json.dumps(dataclasses.asdict(ps.system)), "t": repr(float(t)), "step": str(int(step)),
            "extra": json.dumps(extra or {})}
    save_file(tensors, str(path), metadata=meta)


def read(path):
    """(hierarchy, system, list of CPU U tensors, t, step, extra) from a
    checkpoint file, without touching a device."""
    from safetensors import safe_open
    with safe_open(str(path), framework="pt", device="cpu") as f:
        meta = f.metadata()
        if meta.get("format") != FORMAT:
            raise ValueError(f"{path}: not a {FORMAT} file")
        hier = _hier_from(json.loads(meta["hierarchy"]))
        system = M.System(**json.loads(meta["system"]))
        Us = [f.get_tensor(f"U{l}") for l in range(len(hier.levels))]
    return hier, system, Us, float(meta["t"]), int(meta["step"]), json.loads(meta["extra"])


def restore(path, device: str = "cuda"):
    """Rebuild the patchset and device states of a checkpoint: returns
    (patchset, states, t, step, extra)."""
    hier, system, Us, t, step, extra = read(path)
    ps = M.Patchset(hier, system)
    states = ps.alloc_states(device)
    for l, U in enumerate(Us):
        if U.numel() != ps.layouts[l]["nelems"]:
            raise ValueError(f"level {l}: the file holds {U.numel()} values, the layout {ps.layouts[l]['nelems']}")
        states[l]["U"].copy_(U.reshape(states[l]["U"].shape))
    return ps, states, t, step, extra
