"""Run metrics as JSON lines (one object per ligand and record): the HMC
acceptance of each state and the exchange acceptance of each neighbour pair
(Sampling: the quantities the paper monitors while it adapts a ladder),
replica round trips between the end states, moves rejected for a
non-finite energy, and whatever throughput figures the caller measured
(atom-evals/s, effective GB/s, ESS/s).  Host-side bookkeeping only: every
number comes from the library's counters through the binding."""
from __future__ import annotations

import json
import time


def _ratios(acc, tries):
    return [float(a) / float(t) if t else None for a, t in zip(acc, tries)]


def ligand_metrics(ctx, ligand_id):
    """The counters of one ligand of a Context as a JSON-ready dict."""
    st = ctx.get_stats(ligand_id)
    return {"ligand": int(ligand_id),
            "hmc_acceptance": _ratios(st["hmc_acc"], st["hmc_try"]),
            "exchange_acceptance": _ratios(st["ex_acc"], st["ex_try"]),
            "hmc_tries": int(st["hmc_try"].sum()),
            "exchange_tries": int(st["ex_try"].sum()),
            "round_trips": int(ctx.get_round_trips(ligand_id)),
            "nonfinite": int(st["nonfinite"])}


class MetricsLog:
    """Appends JSON lines to `path`."""

    def __init__(self, path):
        self.path = path

    def write(self, records, **figures):
        """One line per record (a ligand_metrics dict), each with the
        caller's figures (plain JSON values) and a timestamp."""
        with open(self.path, "a") as fh:
            for rec in records:
                line = {"time": time.time(), **rec, **figures}
                fh.write(json.dumps(line) + "\n")

    def record(self, ctx, ligand_ids, **figures):
        """ligand_metrics of every listed ligand, written at once."""
        self.write([ligand_metrics(ctx, i) for i in ligand_ids], **figures)
