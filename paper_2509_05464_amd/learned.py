"""Learned slow-time clutter filter: parameter state, training step, inference.

Orchestration only: the batch gather, forward, backward, Adam update, power Doppler
and the SVD-fallback judge are all HIP kernels behind the C ABI.  The parameters
live on the GPU as FP32 master weights plus the BF16 copy the kernels read.
"""
from __future__ import annotations

from typing import Optional

import numpy as np
import torch

from . import _lib as fq


class LearnedFilter:
    def __init__(self, w0: np.ndarray, device: Optional[torch.device] = None, lr: float = 1e-3):
        device = device or torch.device('cuda')
        w0 = np.ascontiguousarray(w0, dtype=np.float32)
        assert w0.size == fq.LCF_N_PARAM
        self.w = torch.from_numpy(w0.copy()).to(device)
        self.wb = torch.zeros(w0.size, dtype=torch.int16, device=device)
        self.m = torch.zeros_like(self.w)
        self.v = torch.zeros_like(self.w)
        self.grad = torch.zeros_like(self.w)
        # the BF16 copy comes from the Adam kernel: a zero-gradient, zero-rate step
        fq.lcf_adam_step(self.w, self.wb, self.m, self.v, self.grad, 1, lr=0.0)
        self.loss = torch.zeros(1, dtype=torch.float32, device=device)
        self.step = 0
        self.lr = lr
        self.device = device
        self._act = None

    def _act_buf(self, n: int, T: int) -> torch.Tensor:
        need = fq.lcf_act_size(n, T)
        if self._act is None or self._act.numel() < need:
            self._act = torch.empty(need, dtype=torch.uint8, device=self.device)
        return self._act

    def train_step(self, x: torch.Tensor, target: torch.Tensor, eps: float = 1e-30) -> torch.Tensor:
        """One Adam step on a batch: x, target complex64 [T][B] (mix and blood-only series).
        Returns the (device) loss of the batch before the update."""
        T, B = x.shape
        act = self._act_buf(B, T).view(torch.int16)
        fq.lcf_forward(self.w, self.wb, x, eps, act, None, None)
        fq.lcf_backward(self.w, self.wb, x, target, act, self.grad, self.loss, eps)
        self.step += 1
        fq.lcf_adam_step(self.w, self.wb, self.m, self.v, self.grad, self.step, lr=self.lr)
        return self.loss

    def infer(self, iq: torch.Tensor, pd: torch.Tensor, y: Optional[torch.Tensor] = None, eps: float = 1e-30) -> None:
        """Blood estimate of every voxel series of iq (complex64 [T][Nv]) -> pd (and y)."""
        fq.lcf_forward(self.w, self.wb, iq, eps, None, y, pd)

    def state(self) -> dict:
        return {'w': self.w.cpu().numpy(), 'm': self.m.cpu().numpy(), 'v': self.v.cpu().numpy(),
                'step': np.int64(self.step), 'lr': np.float32(self.lr)}

    def save(self, path: str) -> None:
        np.savez(path, **self.state())

    @classmethod
    def load(cls, path: str, device: Optional[torch.device] = None) -> 'LearnedFilter':
        d = np.load(path)
        f = cls(d['w'], device, float(d['lr']))
        f.m.copy_(torch.from_numpy(d['m']))
        f.v.copy_(torch.from_numpy(d['v']))
        f.step = int(d['step'])
        return f


def fallback(pd_learned: torch.Tensor, pd_svd: torch.Tensor, out: torch.Tensor, tau_db: float = -10.0):
    """SVD fallback judge: returns device tensors (flag, d_db); out holds the chosen PD."""
    ws = torch.empty(fq.fallback_workspace_size(pd_learned.numel()), dtype=torch.uint8, device=pd_learned.device)
    flag = torch.zeros(1, dtype=torch.int32, device=pd_learned.device)
    d_db = torch.zeros(1, dtype=torch.float32, device=pd_learned.device)
    fq.lcf_fallback(pd_learned, pd_svd, out, flag, d_db, ws, tau_db)
    return flag, d_db
