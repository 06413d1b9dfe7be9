"""Tiling autotuner for a LloidPlan.

The plan's tiling options (the correlation item's columns and tap split,
how many consecutive correlation and mixing work items share one XCD, and
the order of the mixing items) change how one
stride's work is cut into work groups, never what is computed.  The best
setting depends on the bank mix: many short filters want short tap splits
for enough work groups, long filters want long splits so that the split-K
reduction reads fewer partial planes.

autotune() times each candidate with the plan's own per-kernel HIP-event
profiler on a few strides of the caller's strain, one option at a time
(correlation columns and split, measured by correlation + reduction time;
correlation grouping; mixing grouping and item order), keeps the fastest setting of each, then resets
the plan's stream state so that filtering starts from stride 0.
"""
from __future__ import annotations

from typing import Callable, Optional, Sequence

DEFAULT_COLS = (64, 128, 256, 512)
DEFAULT_SPLITS = (512, 1024, 2048, 4096, 8192)
DEFAULT_CORR_GROUPS = (0, 8, 16, 32)
DEFAULT_MIX_GROUPS = (0, 16, 32, 64, 128, 256)
DEFAULT_MIX_TBLOCKS = (1, 2, 4, 8, 16)


def _time(plan, strides: Sequence, kernels: Sequence[str], write_series: bool) -> float:
    """Mean ms per stride of `kernels`, after one untimed stride."""
    import torch
    series = plan.new_series() if write_series else None
    peaks = plan.new_peaks()
    plan.push(strides[0], series=series, peaks=peaks, write_series=write_series)
    torch.cuda.synchronize()
    plan.profile(True)
    for x in strides[1:]:
        plan.push(x, series=series, peaks=peaks, write_series=write_series)
    torch.cuda.synchronize()
    prof = plan.profile_read()
    plan.profile(False)
    n = max(len(strides) - 1, 1)
    return sum(prof[k][0] for k in kernels) / n


def autotune(plan, strides: Sequence, cols: Sequence[int] = DEFAULT_COLS, splits: Sequence[int] = DEFAULT_SPLITS,
             corr_groups: Sequence[int] = DEFAULT_CORR_GROUPS, mix_groups: Sequence[int] = DEFAULT_MIX_GROUPS,
             mix_tblocks: Sequence[int] = DEFAULT_MIX_TBLOCKS, write_series: bool = True, log: Optional[Callable[[str], None]] = None) -> dict:
    """Tune `plan` on `strides` (device tensors [n_det][F], at least 2).

    Returns {"corr_cols", "corr_split", "corr_group", "mix_group", "mix_tblock", "timings"}; the chosen
    values are left set on the plan, whose stream state is reset."""
    if len(strides) < 2:
        raise ValueError("autotune needs at least two strides")
    timings = {}

    def sweep(option: str, values: Sequence[int], kernels: Sequence[str]) -> int:
        best, best_ms = plan.option(option), None
        for v in values:
            plan.set_option(option, v)
            plan.reset()
            ms = _time(plan, strides, kernels, write_series)
            timings[f"{option}={v}"] = ms
            if log:
                log(f"autotune {option}={v}: {'+'.join(kernels)} {ms:.4f} ms/stride")
            if best_ms is None or ms < best_ms:
                best, best_ms = v, ms
        plan.set_option(option, best)
        return best

    ccols = sweep("corr_cols", cols, ("corr", "reduce"))
    split = sweep("corr_split", splits, ("corr", "reduce"))
    cgroup = sweep("corr_group", corr_groups, ("corr",))
    mgroup = sweep("mix_group", mix_groups, ("mix",))
    tblock = sweep("mix_tblock", mix_tblocks, ("mix",))
    mgroup = sweep("mix_group", mix_groups, ("mix",))   # again, for the chosen item order
    plan.reset()
    return {"corr_cols": ccols, "corr_split": split, "corr_group": cgroup, "mix_group": mgroup,
            "mix_tblock": tblock, "timings": timings}
