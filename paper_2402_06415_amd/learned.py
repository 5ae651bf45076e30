"""Learned whole-lattice proposals: training-data generation, training and
the combined chain (plain sweeps plus one network proposal every k sweeps),
as sequences of libising.so calls on the current stream."""
from __future__ import annotations

import numpy as np

from .binding import Batch, Net, ising_batch_mh


def plain_configurations(L: int, beta: float, chains: int, therm: int, snapshots: int, gap: int,
                         seed: int, device=None):
    """Configurations from the plain sampler: `chains` lattices at beta,
    `therm` sweeps of equilibration, then `snapshots` copies each `gap`
    sweeps apart.  Returns an int8 device tensor [snapshots * chains, L, L]."""
    import torch

    assert (L * L) % 256 == 0, "contiguous lattices need L*L to be a multiple of 256"
    b = Batch([L] * chains, [beta] * chains, seed=seed, start="random", device=device)
    b.sweep(therm, moments=False)
    out = torch.empty((snapshots * chains, L, L), dtype=torch.int8, device=b.device)
    lat = b.spins[:chains * L * L].view(torch.int8).view(chains, L, L)
    for k in range(snapshots):
        b.sweep(gap, moments=False)
        out[k * chains:(k + 1) * chains].copy_(lat)
    return out


def train(net: Net, data, epochs: int, batch: int, lr: float, seed: int = 0):
    """Adam on the mean negative log-likelihood of `data` (int8 device
    tensor [n, L, L]) in shuffled minibatches; returns the loss after each
    step (host numpy)."""
    import torch

    n = data.shape[0]
    g = torch.Generator().manual_seed(seed)
    mb = torch.empty((batch, net.L, net.L), dtype=torch.int8, device=data.device)
    losses = []
    dev_losses = torch.empty(epochs * (n // batch), dtype=torch.float32, device=data.device)
    k = 0
    for _ in range(epochs):
        perm = torch.randperm(n, generator=g).to(data.device)
        for i in range(n // batch):
            torch.index_select(data, 0, perm[i * batch:(i + 1) * batch], out=mb)
            net.loss_and_grad(mb, loss=dev_losses[k:k + 1])
            net.adam(lr)
            k += 1
    losses = dev_losses[:k].cpu().numpy()
    return losses


class LearnedChains:
    """`count` chains of side L at betas: each cycle runs k plain sweeps,
    then proposes a whole new lattice per chain from the network (by
    default Z2-symmetrised: q_sym(s) = (q(s) + q(-s)) / 2) and accepts it
    with the Metropolis-Hastings probability (ising_batch_mh)."""

    def __init__(self, net: Net, L: int, betas, seed: int, lattice_id0: int = 0,
                 sweeps_per_proposal: int = 10, start: str = "random", device=None,
                 symmetric: bool = True):
        import torch

        self.net, self.L, self.k = net, L, sweeps_per_proposal
        self.symmetric = symmetric
        self.count = len(betas)
        assert self.count <= net.max_batch and net.L == L
        self.batch = Batch([L] * self.count, betas, seed=seed, lattice_id0=lattice_id0,
                           start=start, device=device)
        # the sweeps' launch shape, timed on scratch spins (the chain is the
        # same under every shape): the default suits large lattices, and a
        # leaner one also leaves more of each CU to the sampler beside it
        self.batch.autotune()
        dev = self.batch.device
        self.seed, self.lid0 = seed, lattice_id0
        self.beta = torch.as_tensor(np.asarray(betas, np.float64), device=dev)
        self.prop = torch.empty((self.count, L, L), dtype=torch.int8, device=dev)
        self.lq_cur = torch.empty(self.count, dtype=torch.float32, device=dev)
        self.lq_prop = torch.empty(self.count, dtype=torch.float32, device=dev)
        # each cycle's acceptance flags go to a row of a ring, added to the
        # per-chain totals once per ring (one reduction instead of one add
        # per cycle) or when the totals are read
        self._ring = torch.zeros((self._RING, self.count), dtype=torch.int32, device=dev)
        self._rows = 0   # rows written since the last fold
        self._last = self._RING - 1
        self._n = torch.zeros(self.count, dtype=torch.int64, device=dev)
        self.draw = 0
        # the proposals do not depend on the chains' states: the k sweeps
        # run on a second stream (default priority) while the caller's
        # stream draws the proposals
        self.side = torch.cuda.Stream(device=dev)

    _RING = 64

    @property
    def accepted(self):
        """The last cycle's acceptance flags (int32 per chain, device)."""
        return self._ring[self._last]

    @property
    def n_accepted(self):
        """Accepted proposals per chain since construction or the last
        zero_() of this tensor (int64, device)."""
        self._fold()
        return self._n

    def _fold(self):
        if self._rows:
            self._n += self._ring[:self._rows].sum(0)
            self._rows = 0

    def cycle(self, trace=None):
        """k sweeps (E, M after each into trace [k, count, 2] if given), then one proposal."""
        import torch

        main = torch.cuda.current_stream()
        # the sweeps follow the previous cycle's acceptance step
        self.side.wait_stream(main)
        with torch.cuda.stream(self.side):
            self.batch.sweep(self.k, moments=False, trace=trace)
        # the sampler's log q is bitwise the one logq() would give the proposal
        self.net.sample(self.count, self.seed, chain0=self.lid0, draw=self.draw, out=self.prop,
                        logq=self.lq_prop, symmetric=self.symmetric)
        main.wait_stream(self.side)
        self.net.logq(self.batch, out=self.lq_cur, symmetric=self.symmetric)
        if self._rows == self._RING:
            self._fold()
        row = self._ring[self._rows]
        ising_batch_mh(self.batch.c, self.L, self.prop.data_ptr(), self.L * self.L,
                       self.lq_cur.data_ptr(), self.lq_prop.data_ptr(), self.beta.data_ptr(),
                       self.draw, row.data_ptr(), torch.cuda.current_stream().cuda_stream)
        self._last = self._rows
        self._rows += 1
        self.draw += 1
