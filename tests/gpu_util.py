"""Helpers for the GPU parity tests (oracle on the CPU, library on the GPU)."""
import os
import sys

import numpy as np
import pytest
import torch


def require_gpu():
    if not torch.cuda.is_available():
        pytest.fail("a GPU test was selected but no GPU is visible")


def announce(*parts):
    print("[case]", *parts, flush=True)
    sys.stdout.flush()


def to_dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def rel_err(got, want):
    got = got.detach().cpu().numpy() if isinstance(got, torch.Tensor) else got
    scale = np.max(np.abs(want))
    return float(np.max(np.abs(got - want)) / (scale if scale > 0 else 1.0))


class engine_path:
    """Force the four-step path for 1D plans created inside the block."""
    def __enter__(self):
        os.environ["AZRBF_ENGINE"] = "1"

    def __exit__(self, *a):
        os.environ.pop("AZRBF_ENGINE", None)


def oracle_norms(prob, tauZ=1e-12):
    """||A^c||_2 and ||Z*||_2 from the oracle's symbol D = sum_r |d_r|^2 of the
    periodic operator (Lemma 4.2): the singular values of A^c are sqrt(D) and
    those of the regularised Z* are 1/sqrt(D) on the kept modes (closed form
    for 1D approximation, from the sampled kernel otherwise)."""
    from oracle import periodic, spectra
    if prob.dim == 1 and prob.op == 0:
        D = sum(np.abs(spectra.diag_closed_form(prob.n, prob.s, prob.T, prob.eps, r)) ** 2 for r in range(prob.s))
    else:
        _, D = periodic.symbol_weights(prob, tauZ)
    keep = D > tauZ * D.max()
    return float(np.sqrt(D.max())), float(1.0 / np.sqrt(D[keep].min()))
