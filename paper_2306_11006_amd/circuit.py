"""Levelled evaluation of a gate DAG on the GPU (ArctyrEX Section 4.2).

The netlist is levelised once on the host by the library's Kahn pass
(cggi_levelize); each level becomes one device array of gate descriptors and
is evaluated by one cggi_eval_level call.  `capture` records every level of
the circuit into one HIP graph (through torch.cuda.CUDAGraph) so a replay
costs a single launch from the host.
"""
import numpy as np
import torch

from . import cggi


class LevelledCircuit:
    def __init__(self, gates, n_wires, device="cuda"):
        gates = np.ascontiguousarray(gates, dtype=np.int32).reshape(-1, 5)
        self.gates = gates
        self.n_wires = int(n_wires)
        order, start = cggi.levelize(gates, self.n_wires)
        self.order = order
        self.level_start = start
        self.levels = [gates[order[start[i]:start[i + 1]]]
                       for i in range(len(start) - 1)]
        self.d_levels = [cggi.to_device(lv, device) for lv in self.levels]
        self.widths = [len(lv) for lv in self.levels]
        self.level_bootstraps = [self._bootstraps(lv) for lv in self.levels]

    @property
    def n_levels(self):
        return len(self.levels)

    @staticmethod
    def _bootstraps(gates):
        ops = gates[:, 0]
        return int(np.isin(ops, (0, 1, 2, 3, 9, 10)).sum() +
                   2 * (ops == 4).sum())

    def bootstraps(self):
        return self._bootstraps(self.gates)

    def forms_for(self, form, table=None):
        """The form of each level: `form` itself, or for form == "auto" the
        faster one at the level's bootstrap count in an autotuner table
        (paper_2306_11006_amd.tune)."""
        if form != "auto":
            return [form] * self.n_levels
        from .tune import best_form
        return [best_form(table or {}, b) for b in self.level_bootstraps]

    def run(self, ctx, form, wires, stream=None, table=None):
        ctx.reserve(max(self.widths) if self.widths else 0)
        for lv, f in zip(self.d_levels, self.forms_for(form, table)):
            ctx.eval_level(f, lv, wires, stream=stream)
        return wires

    def capture(self, ctx, form, wires, table=None):
        """Record all levels into one graph; replay with graph.replay().
        The workspace is reserved first, so nothing is allocated inside."""
        ctx.reserve(max(self.widths) if self.widths else 0)
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        torch.cuda.synchronize()
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph, stream=side):
            for lv, f in zip(self.d_levels, self.forms_for(form, table)):
                ctx.eval_level(f, lv, wires)
        return graph
