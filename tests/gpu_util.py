"""Helpers for the GPU parity tests: seeded inputs, layout conversion through the
oracle's own converter, and the relative-RMS metric."""
from __future__ import annotations

import sys

import numpy as np

import oracle
from paper_2208_10154_amd import synth


def note(msg: str) -> None:
    """Name the case before any GPU step (so a fault can be attributed)."""
    print(f"[gpu-case] {msg}", flush=True)
    sys.stdout.flush()


def rel_rms(x: np.ndarray, ref: np.ndarray, axis=-1) -> np.ndarray:
    """||x - ref||_2 / ||ref||_2 along `axis` (per map and component)."""
    num = np.sqrt(np.sum((x - ref) ** 2, axis=axis))
    den = np.sqrt(np.sum(ref ** 2, axis=axis))
    return num / np.where(den == 0, 1.0, den)


def alm_inputs(lmax: int, nmaps: int, pol: bool, workload: int, first: int = 0):
    """(complex oracle-format alm [n, (3,) L+1, L+1], compact float64 [n, ncomp, (L+1)^2])."""
    a = synth.gaussian_alm(lmax, nmaps, pol, workload, first)
    if not pol:
        a = a[:, None]
    return a, oracle.to_compact(a)


def to_dev(x: np.ndarray):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def from_dev(t) -> np.ndarray:
    return t.detach().cpu().numpy()
