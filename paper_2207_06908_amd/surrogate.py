"""Learned surrogate of the electrode sweep, with FDTD as fallback and judge.

A case is a buried horizontal electrode (Section 4.1 feed arrangement) in a
homogeneous soil, described by five inputs: log10 of the soil conductivity,
its relative permittivity, the electrode length and depth, and the front
time T1 of the injected 1 A double-exponential current (T2 = 10 us).  Its
answer is the ground potential rise (GPR) at the feed over 2000 steps of the
dx = 0.25 m grid (0.953 us), resampled to 256 points.

* Dataset: cases are simulated by the batched FDTD engine (one launch per
  step over all grids of a chunk, HIP-graph replay).  Every case runs on a
  grid whose size follows from the case alone (the electrode length sets
  nx), so a case has exactly one FDTD answer.  Length and depth are taken at
  the grid resolution, as the engine sees them.
* Network: 5 -> 512 x 4 (GELU) -> 256, trained by the BF16-MFMA kernels of
  the surrogate library with Adam.  Targets are the GPR divided by a
  closed-form resistance scale of the electrode (a horizontal-electrode
  resistance formula with the soil's conductivity augmented by its
  displacement-current term eps / T1), which removes most of the three
  decades of amplitude range.
* Routing: an ensemble of independently seeded nets answers every query in
  one batched inference; a query whose nets disagree on the GPR peak by more
  than a threshold (spread (max - min) / |mean|) goes to the FDTD engine.

All numerical work runs in the HIP library; this module prepares inputs,
drives the calls and evaluates errors.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, replace
from typing import List, Sequence

import numpy as np

from . import scenarios as S

WIDTHS = [5, 512, 512, 512, 512, 256]
N_OUT = 256
N_STEPS = 2000
DX = 0.25
NPML = 8
T2 = 10e-6
WIRE_RADIUS = 0.005
RANGES = S.CONFIG3_RANGES
EPS0 = 1.0 / (4e-7 * math.pi * S.C0 ** 2)  # vacuum permittivity, only for the target scale
# Operating points of the routing.  FAST: spread > 2% goes to FDTD.  GUARDED:
# also every query outside the training box (bound 1 on the scaled inputs,
# with room for the float rounding of inputs on the box faces), with a 0.5%
# spread threshold.
FAST_THRESHOLD = 0.02
GUARD_BOUND = 1.0 + 1e-5
GUARD_THRESHOLD = 0.005


# ---------------------------------------------------------------------------
# Cases, grids and source waveforms
# ---------------------------------------------------------------------------

def quantize(case: S.ElectrodeCase, dx: float = DX) -> S.ElectrodeCase:
    """Length and depth at the grid resolution (what the FDTD grid holds)."""
    return replace(case, length=max(1, round(case.length / dx)) * dx,
                   depth=max(1, round(case.depth / dx)) * dx)


def canonical_dims(case: S.ElectrodeCase, dx: float = DX):
    """Grid size determined by the case: 48 x 48 cells across, x long enough
    for the electrode, the feed stubs and the absorbing layer."""
    n_w = int(round(case.length / dx))
    return max(48, n_w + 24), 48, 48


class SourceTable:
    """Double-exponential parameters (alpha, beta) as smooth functions of T1
    for fixed T2: exact solves at nodes, cubic interpolation of log alpha and
    log beta in between (relative error below 1e-6 in T1 over the table)."""

    def __init__(self, t2: float = T2, lo: float = 0.35e-6, hi: float = 1.65e-6, n: int = 53):
        from scipy.interpolate import CubicSpline
        self.t2, self.lo, self.hi = t2, lo, hi
        self.nodes = np.linspace(lo, hi, n)
        ab = np.array([S.dexp_params(t1, t2)[:2] for t1 in self.nodes])
        self._la = CubicSpline(self.nodes, np.log(ab[:, 0]))
        self._lb = CubicSpline(self.nodes, np.log(ab[:, 1]))

    def params(self, t1: float):
        if not (self.lo <= t1 <= self.hi):
            raise ValueError(f"T1 {t1:.3e} s outside the source table")
        a, b = math.exp(float(self._la(t1))), math.exp(float(self._lb(t1)))
        tp = math.log(b / a) / (b - a)
        k = 1.0 / (math.exp(-a * tp) - math.exp(-b * tp))
        return a, b, k

    def waveform(self, t1: float, n_steps: int, dt: float) -> np.ndarray:
        a, b, k = self.params(t1)
        t = S.sample_times(n_steps, dt)
        return k * (np.exp(-a * t) - np.exp(-b * t))


_TABLE = None


def source_table() -> SourceTable:
    global _TABLE
    if _TABLE is None:
        _TABLE = SourceTable()
    return _TABLE


def case_scenario(case: S.ElectrodeCase, n_steps: int = N_STEPS, name: str = "case") -> S.Scenario:
    """The FDTD scenario of a (quantized) case on its canonical grid."""
    case = quantize(case)
    amps = source_table().waveform(case.T1, n_steps, S.courant_dt(DX))
    return S.electrode_grid(case, canonical_dims(case), dx=DX, npml=NPML, n_steps=n_steps, T2=T2, name=name,
                            amps=amps)


# ---------------------------------------------------------------------------
# Features and targets
# ---------------------------------------------------------------------------

def _conductance(log10_sigma: float, eps_r: float, T1: float) -> float:
    """Conduction plus displacement conductivity at the front time scale,
    sigma + eps0 eps_r / T1 (S/m)."""
    return 10.0 ** log10_sigma + EPS0 * eps_r / T1


def _feature_box():
    """Ranges of the five inputs over the corners of the training box."""
    (s0, s1), (e0, e1), (t0, t1) = RANGES["log10_sigma"], RANGES["eps_r"], RANGES["T1"]
    return [(math.log10(_conductance(s0, e0, t1)), math.log10(_conductance(s1, e1, t0))),
            (10.0 ** s0 / _conductance(s0, e1, t0), 10.0 ** s1 / _conductance(s1, e0, t1)),
            RANGES["length"], RANGES["depth"], RANGES["T1"]]


FEATURE_BOX = _feature_box()


def features(cases: Sequence[S.ElectrodeCase]) -> np.ndarray:
    """The network inputs of (quantized) cases: log10 of the conductance
    g = sigma + eps0 eps_r / T1, the conduction fraction sigma / g, length,
    depth and T1, each scaled so that the training box maps into [-1, 1].
    (sigma, eps_r) and (g, sigma / g) carry the same information for a given
    T1; the second pair keeps queries outside the training ranges of sigma
    and eps_r nearer the box, where the nets of the ensemble agree better.)"""
    out = np.empty((len(cases), 5), np.float32)
    for n, c in enumerate(map(quantize, cases)):
        g = _conductance(c.log10_sigma, c.eps_r, c.T1)
        vals = (math.log10(g), 10.0 ** c.log10_sigma / g, c.length, c.depth, c.T1)
        for q, (v, (lo, hi)) in enumerate(zip(vals, FEATURE_BOX)):
            out[n, q] = 2.0 * (v - lo) / (hi - lo) - 1.0
    return out


def resistance_scale(cases: Sequence[S.ElectrodeCase]) -> np.ndarray:
    """rho_eff / (pi L) (ln(2L / sqrt(2 a d)) - 1) with 1/rho_eff = sigma +
    eps0 eps_r / T1: the resistance of a horizontal electrode of length L,
    radius a, depth d, with the displacement current at the front time scale
    added to the conduction current."""
    out = np.empty(len(cases))
    for n, c in enumerate(map(quantize, cases)):
        g = 10.0 ** c.log10_sigma + EPS0 * c.eps_r / c.T1
        out[n] = (math.log(2.0 * c.length / math.sqrt(2.0 * WIRE_RADIUS * c.depth)) - 1.0) / (math.pi * c.length * g)
    return out


def resample(v: np.ndarray, n_out: int = N_OUT) -> np.ndarray:
    """Linear interpolation of waveforms [n, n_steps] (sample s at (s+1) dt)
    at the n_out times (j + 1) T / n_out, T = n_steps dt."""
    n_steps = v.shape[-1]
    src = np.arange(1, n_steps + 1, dtype=np.float64)
    dst = np.arange(1, n_out + 1, dtype=np.float64) * (n_steps / n_out)
    return np.stack([np.interp(dst, src, row) for row in np.atleast_2d(v)])


def gpr_from_probe(v_gap: np.ndarray) -> np.ndarray:
    """The voltage-gap probe integrates E along +y from the remote lead to the
    electrode's riser, i.e. minus the potential rise of the electrode."""
    return -v_gap


def peak_error(pred: np.ndarray, ref: np.ndarray) -> np.ndarray:
    """|max(pred) - max(ref)| / |max(ref)| per row."""
    pp, pr = pred.max(axis=-1), ref.max(axis=-1)
    return np.abs(pp - pr) / np.abs(pr)


def l2_error(pred: np.ndarray, ref: np.ndarray) -> np.ndarray:
    return np.linalg.norm(pred - ref, axis=-1) / np.linalg.norm(ref, axis=-1)


# ---------------------------------------------------------------------------
# FDTD side
# ---------------------------------------------------------------------------

@dataclass
class FdtdRun:
    gpr: np.ndarray        # [n, n_steps] volts per ampere
    gpu_ms: float          # event time of the batched steps
    wall_s: float          # set-up + steps + probe read-back
    cells: int


def run_fdtd(cases: Sequence[S.ElectrodeCase], n_steps: int = N_STEPS, chunk: int = 2048,
             graph_steps: int = 100, log=None) -> FdtdRun:
    """GPR of every case from the batched FDTD engine: at most `chunk` grids
    per batch, the batches of equal size (a small last batch would leave
    the device half idle)."""
    import torch
    from . import fdtd
    out = np.zeros((len(cases), n_steps))
    gpu_ms, cells = 0.0, 0
    t0 = time.perf_counter()
    n_chunks = max(1, -(-len(cases) // chunk))
    chunk = -(-len(cases) // n_chunks) if cases else chunk
    for c0 in range(0, len(cases), chunk):
        part = cases[c0:c0 + chunk]
        grids, pids = [], []
        for q, case in enumerate(part):
            sc = case_scenario(case, n_steps, name=f"case{c0 + q}")
            g = fdtd.Grid.from_params(sc.params(), precision=32)
            ids = S.apply(sc, g)
            pids.append(ids[[p[0] for p in sc.probes].index("V_gap")])
            grids.append(g)
        # two-step 60 x 8 tiles: the batched engine's fastest shape on these grids
        g_steps = graph_steps if n_steps % graph_steps == 0 and graph_steps % 4 == 0 else 0
        b = fdtd.Batch(grids, tile=(60, 8, 32), graph_steps=g_steps)
        b.bind()
        b.timing(True)
        b.run(n_steps)
        ms, _n = b.time()
        b.timing(False)
        gpu_ms += ms
        cells += b.cells
        for q in range(len(part)):
            out[c0 + q] = gpr_from_probe(b.probe(q, pids[q]))
        del b, grids
        torch.cuda.empty_cache()
        if log:
            log(f"fdtd chunk {c0 // chunk}: {len(part)} cases, {ms:.0f} ms on the GPU")
    return FdtdRun(out, gpu_ms, time.perf_counter() - t0, cells)


# ---------------------------------------------------------------------------
# Network side
# ---------------------------------------------------------------------------

class Surrogate:
    """Ensemble of MLPs on the GPU (surrogate library)."""

    def __init__(self, n_nets: int = 4, max_rows: int = 8192, widths=WIDTHS):
        from . import sur
        self.widths = list(widths)
        self.n_nets = n_nets
        self.ens = sur.Ensemble(self.widths, n_nets=n_nets, max_rows=max_rows)

    def init(self, seeds: Sequence[int]):
        for q, s in enumerate(seeds):
            self.ens.init_params(q, int(s))

    def train(self, X: np.ndarray, Y: np.ndarray, epochs: int = 50, batch: int = 1024, lr: float = 1e-3,
              lr_min: float = 1e-5, seed: int = 0, log=None):
        """Adam on shuffled mini-batches (every net its own shuffle), the
        learning rate following a cosine from lr to lr_min over the run.
        Targets are standardised per output during training; the scale and
        offset are folded into the last layer afterwards, so the nets then
        answer in the units of Y.  Returns per-net mean epoch losses (in
        standardised units)."""
        import torch
        dev = self.ens.device
        mu = Y.mean(axis=0).astype(np.float64)
        sd = Y.std(axis=0).astype(np.float64)
        sd = np.maximum(sd, 1e-3 * sd.max())
        Yn = (Y - mu) / sd
        xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(dev)
        yd = torch.from_numpy(np.ascontiguousarray(Yn, np.float32)).to(dev)
        n = X.shape[0]
        rng = np.random.default_rng(seed)
        nb = (n + batch - 1) // batch
        total = epochs * nb
        losses = torch.zeros((self.n_nets, epochs, nb), dtype=torch.float32, device=dev)
        for ep in range(epochs):
            for q in range(self.n_nets):
                perm = torch.from_numpy(rng.permutation(n).astype(np.int32)).to(dev)
                for bi in range(nb):
                    t = ep * nb + bi
                    lr_t = lr_min + 0.5 * (lr - lr_min) * (1.0 + math.cos(math.pi * t / total))
                    rows = perm[bi * batch:(bi + 1) * batch]
                    self.ens.train_step(q, xd, yd, rows=rows, lr=lr_t, loss=losses[q, ep, bi:bi + 1])
            if log and (ep % 10 == 9 or ep == epochs - 1):
                log(f"epoch {ep + 1}: loss " + " ".join(f"{v:.3e}" for v in losses[:, ep].mean(1).tolist()))
        for q in range(self.n_nets):
            self._fold_output_scale(q, mu, sd)
        return losses.mean(2).cpu().numpy()

    def _fold_output_scale(self, net: int, mu: np.ndarray, sd: np.ndarray):
        """y = sd * (W a + b) + mu  ->  W' = diag(sd) W, b' = sd b + mu."""
        flat = self.ens.get_params(net).astype(np.float64)
        k, n = self.widths[-2], self.widths[-1]
        ob = flat.size - n
        ow = ob - n * k
        W = flat[ow:ob].reshape(n, k)
        flat[ow:ob] = (sd[:, None] * W).ravel()
        flat[ob:] = sd * flat[ob:] + mu
        self.ens.set_params(net, flat.astype(np.float32))

    def predict(self, X: np.ndarray, net: int = 0) -> np.ndarray:
        import torch
        xd = torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(self.ens.device)
        return self.ens.forward(net, xd).cpu().numpy()

    def route(self, X, threshold: float = 0.02):
        """(mean prediction, spread, fallback row ids) -- device tensors in, host arrays out."""
        import torch
        xd = X if isinstance(X, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(X, np.float32)).to(
            self.ens.device)
        ym, sp, ids, cnt = self.ens.infer_route(xd, threshold)
        n = int(cnt.item())
        return ym.cpu().numpy(), sp.cpu().numpy(), ids[:n].cpu().numpy()

    def guard(self, bound: float = GUARD_BOUND):
        """Send every query outside the training box (an input beyond
        +-bound after scaling) to the fallback; math.inf switches it off."""
        self.ens.set_input_bound(bound)

    def save(self, path: str):
        """Weights as bfloat16 (the precision the products use), biases FP32."""
        import torch
        arrs = {}
        for q in range(self.n_nets):
            flat = self.ens.get_params(q)
            off = 0
            for l, (k, n) in enumerate(zip(self.widths[:-1], self.widths[1:])):
                W = torch.from_numpy(flat[off:off + n * k].copy()).to(torch.bfloat16)
                arrs[f"net{q}_W{l}"] = W.view(torch.int16).numpy()
                off += n * k
                arrs[f"net{q}_b{l}"] = flat[off:off + n].copy()
                off += n
        np.savez_compressed(path, widths=np.array(self.widths), **arrs)

    def load(self, path: str):
        import torch
        d = np.load(path)
        assert list(d["widths"]) == self.widths
        for q in range(self.n_nets):
            parts = []
            for l in range(len(self.widths) - 1):
                W = torch.from_numpy(d[f"net{q}_W{l}"]).view(torch.bfloat16).to(torch.float32).numpy()
                parts += [W.ravel(), d[f"net{q}_b{l}"]]
            self.ens.set_params(q, np.concatenate(parts).astype(np.float32))


def gpr_from_prediction(y: np.ndarray, cases: Sequence[S.ElectrodeCase]) -> np.ndarray:
    """Network outputs (scaled waveforms) back to volts per ampere."""
    return y * resistance_scale(cases)[:, None]
