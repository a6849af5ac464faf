"""Training drivers of the search's networks (pdx_mlp_*): the learned
probe budget and the learned prune bound.

Probe budget.

After START the network decides, for every r = 1 .. nprobe-1, whether a
query of the IVF search may stop after r buckets; the query probes the
smallest accepted r.  It learns from traces the search itself records:

* a traced search (every probed bucket scanned, ADSampling as deployed)
  writes, per query, the network's 72 inputs for each r and the number of
  buckets the result needed (1 + the largest probe rank holding one of its
  ids);
* label of (query, r) = 1 ("stopping after r buckets loses nothing")
  iff r >= that number, i.e. no vector of a later bucket is in the result;
* training: Adam on minibatches of the shuffled samples, forward, backward
  and update in the library's kernels; negatives weighted by w0 because a
  wrong stop costs recall while a late stop only costs time.

The IVF search of Section 2.1 with the ADSampling test of Section 2.3 stays
the fallback: a query the network never stops is searched exactly as
without it.

Prune bound.  ADSampling drops a vector of a bucket after c1 dimensions
when partial * D/c1 > tau_now * (1 + eps0/sqrt(c1))^2 with one eps0 for
every query and bucket.  The network gives each (query, bucket of probe
rank r >= 1) its own eps.  A search exact within the probed buckets
(eps0 = +inf) records, for every returned neighbour outside the START
bucket, the network's inputs and the smallest eps that keeps that neighbour
at every test point, max over c1 of (sqrt(partial * D / (c1 tau_k)) - 1)
sqrt(c1): the running threshold never falls below the final k-th distance
tau_k, so any eps at or above it keeps the neighbour.  The network is
fitted to a high quantile of that target (pinball loss), which keeps about
that share of the true neighbours while bounding each (query, bucket) as
tightly as its statistics allow; a scale applied at search time trades
speed for recall like eps0 does.

Sample selection and shuffling are plain tensor operations; every
forward, backward and update of the networks runs in the library's
kernels.
"""
from __future__ import annotations

from typing import Dict, Optional, Tuple

import numpy as np
import torch

from . import _lib
from .api import MlpState, PdxIndex, ivf_test_points, pdx_search_ivf


def stop_traces(index: PdxIndex, q: torch.Tensor, k: int, nprobe: int, eps0: float = 2.1, **schedule
                ) -> Tuple[torch.Tensor, torch.Tensor, Dict[str, float]]:
    """Traced search of queries q; returns (features [nq * (nprobe-1), 72]
    float32 device, labels [nq * (nprobe-1)] float32 device, stats)."""
    if nprobe < 2:
        raise ValueError("nprobe must be at least 2")
    nq = q.shape[0]
    tf = torch.empty((nq, nprobe, _lib.MLP_IN), dtype=torch.float32, device=q.device)
    need = torch.empty(nq, dtype=torch.int32, device=q.device)
    pdx_search_ivf(index, q, k, nprobe, eps0=eps0, trace=(tf, need), **schedule)
    r = torch.arange(1, nprobe, device=q.device, dtype=torch.int32)
    y = (r[None, :] >= need[:, None]).to(torch.float32)  # [nq, nprobe-1]
    feats = tf[:, : nprobe - 1].reshape(-1, _lib.MLP_IN).contiguous()
    nh = need.cpu().numpy()
    stats = {"samples": int(y.numel()), "positive_rate": float(y.mean().item()),
             "mean_buckets_needed": float(nh.mean()),
             "needed_quantiles": {str(p): float(np.quantile(nh, p)) for p in (0.5, 0.9, 0.95, 0.99)}}
    return feats, y.reshape(-1).contiguous(), stats


def prune_traces(index: PdxIndex, q: torch.Tensor, k: int, nprobe: int, delta_d: int = 0, **schedule
                 ) -> Tuple[torch.Tensor, torch.Tensor, Dict[str, float]]:
    """Search of queries q exact within the probed buckets, recording the
    prune network's samples; returns (features [m, 72] float32 device,
    targets [m] float32 device, stats) over the m samples that exist."""
    if nprobe < 2:
        raise ValueError("nprobe must be at least 2")
    nq = q.shape[0]
    npt = ivf_test_points(index.d, delta_d)
    if npt == 0:
        raise ValueError("no prune tests: delta_d covers every dimension")
    pf = torch.empty((nq, k, _lib.MLP_IN), dtype=torch.float32, device=q.device)
    pt = torch.empty((nq, k), dtype=torch.float32, device=q.device)
    pdx_search_ivf(index, q, k, nprobe, eps0=float("inf"), delta_d=delta_d, prune_trace=(pf, pt), **schedule)
    keep = torch.isfinite(pt.reshape(-1))
    feats = pf.reshape(-1, _lib.MLP_IN)[keep].contiguous()
    targets = pt.reshape(-1)[keep].contiguous()
    t = targets.cpu().numpy()
    stats = {"samples": int(t.size), "test_points": npt,
             "target_quantiles": {str(p): float(np.quantile(t, p)) for p in (0.5, 0.9, 0.99)} if t.size else {}}
    return feats, targets, stats


def initial_theta(seed: int = 0) -> np.ndarray:
    """He-scaled Gaussian weights, zero biases, in the parameter layout
    W1 [64][72] | b1 | W2 [64][64] | b2 | w3 | b3 (padded to 8960)."""
    rng = np.random.default_rng(seed)
    f, h = _lib.MLP_IN, 64
    th = np.zeros(_lib.MLP_PARAMS, dtype=np.float32)
    o = 0
    th[o:o + h * f] = rng.standard_normal(h * f) * np.sqrt(2.0 / f)
    o += h * f + h
    th[o:o + h * h] = rng.standard_normal(h * h) * np.sqrt(2.0 / h)
    o += h * h + h
    th[o:o + h] = rng.standard_normal(h) * np.sqrt(1.0 / h)
    return th


def train_stop_network(feats: torch.Tensor, labels: torch.Tensor, steps: int = 2000, batch: int = 4096,
                       lr: float = 2e-3, w0: float = 4.0, seed: int = 0,
                       stream: Optional[torch.cuda.Stream] = None) -> Tuple[MlpState, Dict[str, float]]:
    """Adam on minibatches of the shuffled samples; returns the trained
    state and the first / last minibatch loss."""
    n = feats.shape[0]
    if n == 0:
        raise ValueError("no training samples")
    perm = torch.from_numpy(np.random.default_rng(seed).permutation(n)).to(feats.device)
    x = feats.index_select(0, perm).contiguous()
    y = labels.index_select(0, perm).contiguous()
    st = MlpState(torch.from_numpy(initial_theta(seed)).to(feats.device), stream=stream)
    loss = torch.empty(1, dtype=torch.float32, device=feats.device)
    b = min(batch, n)
    first = last = None
    for step in range(1, steps + 1):
        lo = ((step - 1) * b) % n
        hi = min(lo + b, n)
        st.train_step(x[lo:hi], y[lo:hi], w0, lr, step, loss=loss, stream=stream)
        if step == 1:
            first = float(loss.item())
    last = float(loss.item())
    return st, {"steps": steps, "batch": b, "lr": lr, "w0": w0, "loss_first": first, "loss_last": last}


def train_prune_network(feats: torch.Tensor, targets: torch.Tensor, steps: int = 2000, batch: int = 4096,
                        lr: float = 2e-3, level: float = 0.95, seed: int = 0, calibrate: bool = True,
                        stream: Optional[torch.cuda.Stream] = None) -> Tuple[MlpState, Dict[str, float]]:
    """Adam on minibatches of the shuffled samples with the pinball loss at
    `level`: the output estimates that quantile of the target given the
    inputs.  With `calibrate`, the output bias is then shifted by the
    level-quantile of the residuals (target - output) over all samples, so
    that exactly that share of the training targets lies at or below the
    output (Adam at a fixed rate leaves the bias oscillating around it).
    Returns the trained state and the first / last minibatch loss."""
    n = feats.shape[0]
    if n == 0:
        raise ValueError("no training samples")
    perm = torch.from_numpy(np.random.default_rng(seed).permutation(n)).to(feats.device)
    x = feats.index_select(0, perm).contiguous()
    y = targets.index_select(0, perm).contiguous()
    st = MlpState(torch.from_numpy(initial_theta(seed)).to(feats.device), stream=stream)
    loss = torch.empty(1, dtype=torch.float32, device=feats.device)
    b = min(batch, n)
    first = None
    for step in range(1, steps + 1):
        lo = ((step - 1) * b) % n
        hi = min(lo + b, n)
        st.train_step(x[lo:hi], y[lo:hi], level, lr, step, loss=loss, kind="pinball", stream=stream)
        if step == 1:
            first = float(loss.item())
    last = float(loss.item())
    info = {"steps": steps, "batch": b, "lr": lr, "level": level, "loss_first": first, "loss_last": last}
    if calibrate:
        resid = (y - st.forward(x, stream=stream)).float()
        kth = max(1, min(n, int(np.ceil(level * n))))
        shift = float(torch.kthvalue(resid.cpu(), kth).values)
        theta = st.theta(stream=stream)
        theta[_B3] += shift
        st = MlpState(theta, stream=stream)
        info["bias_shift"] = shift
    return st, info


_B3 = 64 * 72 + 64 + 64 * 64 + 64 + 64  # index of the output bias in the parameter vector


def save_theta(state: MlpState, path: str) -> None:
    """Parameters as 8960 little-endian float32 values."""
    state.theta().cpu().numpy().astype("<f4").tofile(path)


def load_theta(path: str, device: str = "cuda") -> MlpState:
    th = np.fromfile(path, dtype="<f4")
    if th.size != _lib.MLP_PARAMS:
        raise ValueError(f"{path}: expected {_lib.MLP_PARAMS} float32 values, found {th.size}")
    return MlpState(torch.from_numpy(th.astype(np.float32)).to(device))
