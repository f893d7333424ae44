"""A batch of independent problems driven through one library handle.

Thin layer over the C ABI (``abi``): it allocates the device buffers of a
batch (states, clocks, end times, status), creates the handle, advances the
batch, and can capture an advance of k steps into a HIP graph.  Every
arithmetic step runs in the library's kernels.
"""

import numpy as np

from . import abi
from . import workloads as W


def initial_state(spec):
    """Nodal initial state of a problem spec (keys: pde, N, ncells, k, phase)."""
    if spec["pde"] == "euler":
        return W.euler_density_wave(spec["ncells"], spec["N"], k=spec.get("k", 1),
                                    phase=spec.get("phase", 0.0), noise=spec.get("noise", 0.0),
                                    seed=spec.get("seed", 0))
    if spec["pde"] == "swe":
        return W.swe_bump_nodal(spec["ncells"], spec["N"])
    raise ValueError(f"unknown pde {spec['pde']!r}")


def state_bytes(spec):
    """Device bytes a problem holds: its state and the library's ping-pong copy."""
    M = 3
    return 2 * spec["ncells"] * (spec["N"] + 1) * M * 8


_PDE = {"euler": abi.PDE_EULER, "swe": abi.PDE_SWE}


class Batch:
    """Problems `specs` on cuda:0 with one handle on `stream` (a torch stream)."""

    def __init__(self, specs, precision=abi.FP64, stream=None, cfl=0.4, states=None):
        import torch
        self.torch = torch
        dev = torch.device("cuda:0")
        self.specs = list(specs)
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        n = len(self.specs)
        init = states if states is not None else [initial_state(s) for s in self.specs]
        # the batch's buffers are allocated and filled on the batch's own
        # stream, so that the handle's work is ordered after the fills and
        # the memory is recycled in that stream's order when the batch is freed
        with torch.cuda.stream(self.stream):
            self.u = [torch.tensor(np.ascontiguousarray(x), device=dev) for x in init]
            self.t = torch.zeros(n, dtype=torch.float64, device=dev)
            self.t_end = torch.full((n,), 1.0e300, dtype=torch.float64, device=dev)
            self.dt = torch.zeros(n, dtype=torch.float64, device=dev)
            self.status = torch.zeros(n, dtype=torch.int32, device=dev)
            # most severe status seen by each problem over all calls (the
            # library reports the status of the last call only)
            self.sticky = torch.zeros(n, dtype=torch.int32, device=dev)
        descs = [abi.pde_desc(_PDE[s["pde"]]) for s in self.specs]
        cfgs = [abi.config(s["N"], s["ncells"], precision=precision, cfl=cfl) for s in self.specs]
        self.h = abi.aderdg_init(descs, cfgs, stream=self.stream.cuda_stream)
        self.graph = None
        self.graph_steps = 0
        self.event = None

    @property
    def dofs(self):
        return sum(s["ncells"] * (s["N"] + 1) * 3 for s in self.specs)

    def step(self, nsteps):
        """Enqueue nsteps steps of every problem (asynchronous); an event
        recorded after them tells when they are done (see ready())."""
        with self.torch.cuda.stream(self.stream):
            abi.aderdg_step(self.h, self.u, self.t, self.t_end, self.dt, self.status, nsteps)
            self.torch.minimum(self.sticky, self.status, out=self.sticky)
            self.event = self.torch.cuda.Event()
            self.event.record(self.stream)

    def ready(self):
        """True once the last enqueued advance has finished (non-blocking)."""
        return self.event is None or self.event.query()

    def capture(self, nsteps):
        """Capture an advance of nsteps steps into a HIP graph.  The state
        pointers must already be bound, so one eager step call runs first."""
        torch = self.torch
        self.step(nsteps)
        self.stream.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=self.stream):
            abi.aderdg_step(self.h, self.u, self.t, self.t_end, self.dt, self.status, nsteps)
            torch.minimum(self.sticky, self.status, out=self.sticky)
        self.graph, self.graph_steps = g, nsteps

    def replay(self):
        with self.torch.cuda.stream(self.stream):
            self.graph.replay()

    def freeze(self, idx):
        """Stop advancing problems idx (their end time becomes their time)."""
        if len(idx):
            # the index tensor is made on the batch's stream too: its copy is
            # then ordered before the kernels that read it, and its memory is
            # not recycled before they have run
            with self.torch.cuda.stream(self.stream):
                ii = self.torch.tensor(list(idx), device=self.t.device)
                self.t_end.index_copy_(0, ii, self.t.index_select(0, ii))

    def sweeps(self, k):
        return abi.aderdg_sweep_count(self.h, k)

    def close(self):
        self.graph = None
        if self.h is not None:
            abi.aderdg_free(self.h)
            self.h = None
