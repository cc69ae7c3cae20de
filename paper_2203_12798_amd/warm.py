"""Learned warm start for the DPar2 iteration: training and use of the set
encoder whose kernels live in libdpar2 (dpar2_warm_*).

Orchestration only: features, targets, the forward and backward passes, the
Adam steps and the assembly of starting factors all run in the library's
kernels, and the labels come from the library's own decompositions; torch
holds the device buffers and concatenates minibatches, and the host solves
the small assignment problems that order each target's components like the
prediction's (R x R per tensor, scipy) before the loss.
"""
import dataclasses

import numpy as np

from . import binding as b


@dataclasses.dataclass
class Sample:
    """One training tensor: tokens (K x NF), targets tH, tV (R x R), tW (K x R)
    (device float32)."""
    tok: object
    tH: object
    tV: object
    tW: object


def features(T, o, ws):
    import torch
    R = o.rank
    tok = torch.empty((T.K, R * (R + 1) // 2), dtype=torch.float32, device="cuda")
    b.warm_features(T, o, ws, tok)
    return tok


def label(T, o, ws, f):
    """Sample of tensor T from factors f (the decomposition in ws)."""
    import torch
    R = o.rank
    tH = torch.empty((R, R), dtype=torch.float32, device="cuda")
    tV = torch.empty_like(tH)
    tW = torch.empty((T.K, R), dtype=torch.float32, device="cuda")
    b.warm_targets(T, o, ws, f, tH, tV, tW)
    return Sample(features(T, o, ws), tH, tV, tW)


class WarmNet:
    """Parameters (flat float32) and Adam state of the set encoder."""

    def __init__(self, rank: int, seed: int = 0):
        import torch
        self.R = R = rank
        self.P = b.warm_param_count(R)
        NF, Wd, RR = R * (R + 1) // 2, b.WARM_WIDTH, R * R
        g = torch.Generator(device="cuda").manual_seed(seed)
        parts = []

        def block(rows, cols, std):
            parts.append((torch.randn(rows * cols, device="cuda", generator=g) * std))

        def bias(n, value=None):
            parts.append(torch.zeros(n, device="cuda") if value is None else value)

        # He initialisation for the ReLU layers, small heads; the H head starts
        # at the identity (H^T H = I) and the V~ head at zero
        block(Wd, NF, (2.0 / NF) ** 0.5)
        bias(Wd)
        block(Wd, Wd, (2.0 / Wd) ** 0.5)
        bias(Wd)
        block(RR, Wd, 0.1 / Wd ** 0.5)
        bias(RR, torch.eye(R, device="cuda").reshape(-1))
        block(RR, Wd, 0.1 / Wd ** 0.5)
        bias(RR)
        block(R, 2 * Wd, 0.1 / Wd ** 0.5)
        bias(R, torch.ones(R, device="cuda"))
        self.theta = torch.cat(parts).contiguous()
        assert self.theta.numel() == self.P
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step = 0

    def _buffers(self, n, ntok):
        import torch
        R = self.R
        f = dict(dtype=torch.float32, device="cuda")
        return (torch.empty((ntok, 4 * b.WARM_WIDTH), **f), torch.empty((n, R, R), **f),
                torch.empty((n, R, R), **f), torch.empty((ntok, R), **f))

    def predict(self, tok):
        """(pH, pV, pW) for one tensor's tokens."""
        act, pH, pV, pW = self._buffers(1, tok.shape[0])
        b.warm_forward(self.R, [0, tok.shape[0]], tok, self.theta, act, pH, pV, pW)
        return pH[0], pV[0], pW

    def loss(self, samples, match: bool = True):
        """Mean loss over samples (three terms), no parameter update; match:
        as in train."""
        import torch
        off, tok, tH, tV, tW = self._batch(samples)
        act, pH, pV, pW = self._buffers(len(samples), tok.shape[0])
        b.warm_forward(self.R, off, tok, self.theta, act, pH, pV, pW)
        if match:
            tH, tV, tW = self._match(off, pV, pW, tH, tV, tW)
        gp = torch.empty((len(samples), self.P), dtype=torch.float32, device="cuda")
        grad = torch.empty(self.P, dtype=torch.float32, device="cuda")
        loss = torch.empty((len(samples), 3), dtype=torch.float32, device="cuda")
        b.warm_backward(self.R, off, tok, self.theta, act, pH, pV, pW, tH, tV, tW, gp, grad, loss)
        return loss.mean(dim=0).cpu().numpy()

    @staticmethod
    def _batch(samples):
        import torch
        off = np.concatenate([[0], np.cumsum([s.tok.shape[0] for s in samples])]).astype(np.int32)
        return (off, torch.cat([s.tok for s in samples]), torch.stack([s.tH for s in samples]),
                torch.stack([s.tV for s in samples]), torch.cat([s.tW for s in samples]))

    def _match(self, off, pV, pW, tH, tV, tW):
        """Targets with their components put in the prediction's order, per
        tensor: the assignment of target components to predicted ones that
        minimises the V~ and W squared errors (weighted as in the loss), an
        R x R assignment problem per tensor solved on the host."""
        import torch
        from scipy.optimize import linear_sum_assignment
        R, n = self.R, len(off) - 1
        pv, tv = pV.cpu().numpy(), tV.cpu().numpy()     # n x R x R, column = component
        pw, tw = pW.cpu().numpy(), tW.cpu().numpy()     # tokens x R
        perm = np.empty((n, R), dtype=np.int64)
        for i in range(n):
            a, c = int(off[i]), int(off[i + 1])
            cost = ((pv[i][:, :, None] - tv[i][:, None, :]) ** 2).sum(axis=0) / (R * R)
            cost += ((pw[a:c][:, :, None] - tw[a:c][:, None, :]) ** 2).sum(axis=0) / ((c - a) * R)
            rows, cols = linear_sum_assignment(cost)
            perm[i, rows] = cols
        P = torch.from_numpy(perm).to(tV.device)
        cols = P[:, None, :].expand(n, R, R)
        tV2 = torch.gather(tV, 2, cols)
        tH2 = torch.gather(torch.gather(tH, 2, cols), 1, P[:, :, None].expand(n, R, R))
        tW2 = torch.gather(tW, 1, torch.from_numpy(np.repeat(perm, np.diff(off), axis=0)).to(tW.device))
        return tH2.contiguous(), tV2.contiguous(), tW2.contiguous()

    def train(self, samples, steps: int, batch: int = 16, lr: float = 1e-3, seed: int = 0, log_every: int = 0,
              match: bool = True):
        """Adam on minibatches drawn (without replacement per epoch) from
        samples; returns the mean loss of each logged step.  match: compare
        each tensor's prediction with its target's components reordered to
        the closest assignment (the targets' component order is a gauge
        choice that need not follow from the tokens)."""
        import torch
        rng = np.random.default_rng(seed)
        order, at, hist = rng.permutation(len(samples)), 0, []
        gp = torch.empty((batch, self.P), dtype=torch.float32, device="cuda")
        grad = torch.empty(self.P, dtype=torch.float32, device="cuda")
        loss = torch.empty((batch, 3), dtype=torch.float32, device="cuda")
        for it in range(steps):
            if at + batch > len(order):
                order, at = rng.permutation(len(samples)), 0
            mb = [samples[i] for i in order[at:at + batch]]
            at += batch
            off, tok, tH, tV, tW = self._batch(mb)
            act, pH, pV, pW = self._buffers(len(mb), tok.shape[0])
            b.warm_forward(self.R, off, tok, self.theta, act, pH, pV, pW)
            if match:
                tH, tV, tW = self._match(off, pV, pW, tH, tV, tW)
            b.warm_backward(self.R, off, tok, self.theta, act, pH, pV, pW, tH, tV, tW, gp[:len(mb)], grad,
                            loss[:len(mb)])
            self.step += 1
            b.warm_adam(self.R, self.theta, grad, self.m, self.v, self.step, lr=lr, grad_scale=1.0 / len(mb))
            if log_every and (it % log_every == 0 or it == steps - 1):
                hist.append(float(loss[:len(mb)].sum(dim=1).mean()))
        return hist

    def init_factors(self, T, o, ws, f):
        """Starting factors for T (compressed in ws) written into f."""
        pH, pV, pW = self.predict(features(T, o, ws))
        b.warm_apply(T, o, ws, pH, pV, pW, f)


def iterations_to(T, o, ws, f, target_fit: float, max_iter: int):
    """Runs up to max_iter iterations from the factors in f on the compressed
    tensor in ws; returns (first t with compressed fitness >= target_fit, or
    None, the fitness trace)."""
    import torch
    et = torch.zeros(max_iter, dtype=torch.float64, device="cuda")
    b.als_step(T, o, f, max_iter, ws, err_trace=et)
    rep = b.report_read(T, o, ws)
    fit = 1.0 - et.cpu().numpy()[:rep["iters"]] / rep["xnorm2"]
    hit = np.nonzero(fit >= target_fit)[0]
    return (int(hit[0]) + 1 if hit.size else None), fit
