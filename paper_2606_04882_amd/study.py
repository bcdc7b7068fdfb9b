"""Reference-solution study of Sec. 6 (homogeneous and two-layer tests).

Every scheme of a family runs on the coarse grid as one shot of a single
batched fd_forward call (one launch per step and stencil variant); the
reference runs on a grid refined r times in space and time (r = 16 in the
paper) with a Taylor cross of radius 8.  Errors are taken on the coarse
nodes and times without copying the reference: fd_error_norms reads the
refined snapshot with strides (r, r nx) and the refined traces with row
stride r nrec from row r - 1 (trace row n holds u^{n+1}, i.e. fine row
r (n + 1) - 1); fd_dispersion reads the same trace view for gamma^F and
gamma^W.  Norm scalings as printed in Sec. 6.1.1: snapshot L1 = sum|e| / h^2,
L2 = sqrt(sum e^2) / h, Linf = max|e|; traces with tau for h.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Dict, List, Optional, Sequence

import numpy as np
import torch

from . import autotune, configs, design
from . import fdwave as F


@dataclass(frozen=True)
class Scheme:
    scheme: str     # weight family of design.weights
    shape: str
    M: int
    N: int = 0

    @property
    def label(self) -> str:
        names = {"taylor": "SpatTE", "specte_theta": "SpecTE-theta", "dispte": "DispTE", "displs": "DispLS",
                 "specls": "SpecLS"}
        shp = {"cross": "Cross", "cross_rhombus": "CrossRb", "cross_square": "CrossSq", "rhombus": "Rhombus",
               "square": "Square"}[self.shape]
        arg = f"({self.M},{self.N})" if self.shape in ("cross_rhombus", "cross_square") else f"({self.M})"
        return f"{names.get(self.scheme, self.scheme)}-{shp}{arg}"


REFERENCE = Scheme("taylor", "cross", 8)


def homogeneous_schemes(Ms: Sequence[int] = range(1, 7)) -> List[Scheme]:
    """SpatTE-Cross(M), SpecTE-theta-Cross(M) and DispTE-CrossRb(M, N), N = 1..M."""
    out = []
    for M in Ms:
        out += [Scheme("taylor", "cross", M), Scheme("specte_theta", "cross", M)]
        out += [Scheme("dispte", "cross_rhombus", M, N) for N in range(1, M + 1)]
    return out


def two_layer_schemes(Ms: Sequence[int] = range(1, 7)) -> List[Scheme]:
    """SpatTE-Cross(M), SpecTE-theta-Cross(M) and DispLS-CrossRb(M, N), N = 1..M."""
    out = []
    for M in Ms:
        out += [Scheme("taylor", "cross", M), Scheme("specte_theta", "cross", M)]
        out += [Scheme("displs", "cross_rhombus", M, N) for N in range(1, M + 1)]
    return out


def _grid(w: configs.Workload, nt: int) -> F.Grid:
    return F.Grid(shape=w.shape, h=w.h, dt=w.dt, nt=nt, nb=w.nb, eta_max=w.eta_max, vmax=w.c_max)


def _register(sc: Scheme, courant: float, C_run: float) -> Optional[int]:
    """Stencil id, or None when the weights or the time step are unstable."""
    try:
        w = design.weights(2, sc.scheme, sc.shape, sc.M, courant, N=sc.N)
        sid = F.fd_weights_set(2, sc.shape, sc.M, w, N=sc.N)
    except (F.FdError, ValueError, ZeroDivisionError, ArithmeticError):
        return None
    return sid if C_run <= F.fd_cfl_limit(sid) else None


def _event_seconds(fn) -> float:
    s = torch.cuda.current_stream()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(s)
    fn()
    b.record(s)
    b.synchronize()
    return a.elapsed_time(b) * 1e-3


def run(w: configs.Workload, wf: configs.Workload, schemes: Sequence[Scheme], nscale: int = 128,
        device: str = "cuda:0", reference: Scheme = REFERENCE, tune: bool = False, time_reference: bool = False) -> Dict:
    """Coarse runs of every scheme against the refined reference: per
    scheme the snapshot and trace error norms and the gamma^F / gamma^W norms
    at the trace receiver, averaged and maximised over the receiver line.
    tune: autotune the reference stencil's tile on the refined grid;
    time_reference: run the reference traces twice and time the second call
    (the first one captures the call's graphs)."""
    dev = torch.device(device)
    r = wf.extra["refine"]
    if (wf.shape[0] - 1) != r * (w.shape[0] - 1) or wf.nt != r * w.nt:
        raise ValueError("the reference workload must refine the coarse one")
    nsnap = w.extra["snap_step"]
    itr = w.extra["trace_rec"]
    # -- reference
    vel_f = torch.tensor(configs.study_model(wf), device=dev)
    rid = _register(reference, wf.courant, wf.courant)
    if rid is None:
        raise RuntimeError("reference stencil is unstable at this Courant number")
    wav_f = torch.tensor(wf.wavelet().astype(np.float32), device=dev)
    rec_f = torch.tensor(wf.rec, device=dev)
    ref_tr = torch.zeros(wf.nt, len(wf.rec), device=dev)
    ref_u = (torch.zeros(wf.shape, device=dev), torch.zeros(wf.shape, device=dev))
    if tune:
        autotune.tune(rid, 2, reference.shape, reference.M, _grid(wf, wf.nt), vel_f, wf.src, nt=40, reps=2,
                      N=reference.N)
    shot = F.Shot(stencil_id=rid, src=wf.src, wavelet=wav_f, rec=rec_f, traces=ref_tr)
    t_tr = _event_seconds(lambda: F.fd_forward(_grid(wf, wf.nt), vel_f, [shot]))
    if time_reference:
        t_tr = _event_seconds(lambda: F.fd_forward(_grid(wf, wf.nt), vel_f, [shot]))
    snap_shot = F.Shot(stencil_id=rid, src=wf.src, wavelet=wav_f, final=ref_u)
    t_sn = _event_seconds(lambda: F.fd_forward(_grid(wf, r * nsnap), vel_f, [snap_shot]))
    del vel_f
    # -- coarse runs, every stable scheme as one shot of a batched call
    vel = torch.tensor(configs.study_model(w), device=dev)
    wav = torch.tensor(w.wavelet().astype(np.float32), device=dev)
    rec = torch.tensor(w.rec, device=dev)
    nrec = len(w.rec)
    stable, rows = [], []
    for sc in schemes:
        sid = _register(sc, w.courant, w.courant)
        rows.append({"scheme": sc.label, "M": sc.M, "N": sc.N, "family": sc.scheme, "shape": sc.shape,
                     "stable": sid is not None})
        if sid is not None:
            stable.append((len(rows) - 1, sid))
    tr = [torch.zeros(w.nt, nrec, device=dev) for _ in stable]
    fin = [(torch.zeros(w.shape, device=dev), torch.zeros(w.shape, device=dev)) for _ in stable]
    t_coarse = 0.0
    if stable:
        shots = [F.Shot(stencil_id=sid, src=w.src, wavelet=wav, rec=rec, traces=t) for (_, sid), t in zip(stable, tr)]
        t_coarse = _event_seconds(lambda: F.fd_forward(_grid(w, w.nt), vel, shots))
        snaps = [F.Shot(stencil_id=sid, src=w.src, wavelet=wav, final=f) for (_, sid), f in zip(stable, fin)]
        t_coarse += _event_seconds(lambda: F.fd_forward(_grid(w, nsnap), vel, snaps))
    # -- metrics on the coarse nodes and times (views of the reference)
    ref_snap = ref_u[1][::r, ::r]
    ref_trc = ref_tr[r - 1::r]
    h, dt = w.h, w.dt
    for (i, _), t, f in zip(stable, tr, fin):
        sn = F.fd_error_norms(f[1], ref_snap).cpu().numpy()
        te = F.fd_error_norms(t[:, itr], ref_trc[:, itr]).cpu().numpy()
        d = F.fd_dispersion(t, ref_trc, dt, nscale)
        ndft, ncwt = d["norm_dft"].cpu().numpy(), d["norm_cwt"].cpu().numpy() if nscale > 0 else None
        rows[i].update({
            "snap_l1": float(sn[0] / h ** 2), "snap_l2": float(math.sqrt(sn[1]) / h), "snap_linf": float(sn[2]),
            "trace_l1": float(te[0] / dt ** 2), "trace_l2": float(math.sqrt(te[1]) / dt), "trace_linf": float(te[2]),
            "trace_gamma_dft": float(ndft[itr]), "rec_gamma_dft_avg": float(ndft.mean()),
            "rec_gamma_dft_max": float(ndft.max())})
        if ncwt is not None:
            rows[i].update({"trace_gamma_cwt": float(ncwt[itr]), "rec_gamma_cwt_avg": float(ncwt.mean()),
                            "rec_gamma_cwt_max": float(ncwt.max())})
    upd_f = float(np.prod(wf.shape))
    return {"study": w.name, "refine": r, "courant": w.courant, "nt": w.nt, "snap_step": nsnap,
            "trace_rec": itr, "nrec": nrec, "nscale": nscale,
            "reference": {"stencil": reference.label, "grid": list(wf.shape), "nt": wf.nt,
                          "tile": list(F.fd_get_tile(rid)), "steps_per_launch": F.fd_get_time_block(rid),
                          "seconds_traces": round(t_tr, 3), "seconds_snapshot": round(t_sn, 3),
                          "gupd_s_traces": round(upd_f * wf.nt / t_tr / 1e9, 1)},
            "coarse_seconds": round(t_coarse, 3), "schemes": rows}


def ranking(result: Dict, M: int, key: str = "trace_gamma_dft") -> List[str]:
    """Scheme labels of radius M ordered from least to most dispersive."""
    rows = [r for r in result["schemes"] if r["M"] == M and r["stable"]]
    return [r["scheme"] for r in sorted(rows, key=lambda r: r[key])]


def homogeneous(refine: int = 16, Ms: Sequence[int] = range(1, 7), nscale: int = 128, device: str = "cuda:0",
                **kw):
    return run(configs.study_homogeneous(1), configs.study_homogeneous(refine), homogeneous_schemes(Ms), nscale,
               device, **kw)


def two_layer(refine: int = 16, Ms: Sequence[int] = range(1, 7), nscale: int = 128, device: str = "cuda:0", **kw):
    return run(configs.study_two_layer(1), configs.study_two_layer(refine), two_layer_schemes(Ms), nscale, device,
               **kw)
