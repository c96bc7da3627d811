"""ORACLE -- test infrastructure only.

Reference gradient of the unrolled weighted sum-product form, written with plain
torch FP64 CPU ops and torch.autograd, plus central finite differences of the C
FP64 forward (spa.c).  The forward follows the same equations as spa.c:

  M^(1)_e   = clamp(R_v)
  E^(t)_e   = 2 atanh( prod_{e' in N(c), e' != e} tanh(M^(t)_e' / 2) )          (Eq. 5)
  M^(t+1)_e = clamp( R_v + sum_{e' in N(v), e' != e} w^(t)_e' E^(t)_e' )         (Eq. 6)
  L_v       = R_v + sum_{e in N(v)} w^(T)_e E^(T)_e                              (Eq. 7)
  loss      = mean_{b,v} [ c softplus(L) + (1 - c) softplus(-L) ]

with every "e' != e" written out as a masked product or sum over a padded
neighbour table (no prefix/suffix or total-minus-self shortcuts).
"""
from __future__ import annotations

import numpy as np
import torch

from . import bce_loss, unrolled

L_MAX = 20.0


def _tables(code):
    """Padded neighbour tables: check slots [m, dc_max] and variable slots [n, dv_max] of edge ids (-1 = none)."""
    rp = np.asarray(code.indptr, dtype=np.int64)
    ci = np.asarray(code.indices, dtype=np.int64)
    m, n = code.m, code.n
    E = int(rp[-1])
    dcs = np.diff(rp)
    chk_tab = -np.ones((m, int(dcs.max())), dtype=np.int64)
    for c in range(m):
        chk_tab[c, : dcs[c]] = np.arange(rp[c], rp[c + 1])
    dvs = np.bincount(ci, minlength=n)
    var_tab = -np.ones((n, max(int(dvs.max()), 1)), dtype=np.int64)
    fill = np.zeros(n, dtype=np.int64)
    for e in range(E):  # ascending edge id == ascending check
        v = ci[e]
        var_tab[v, fill[v]] = e
        fill[v] += 1
    return chk_tab, var_tab, ci, E


def forward_torch(code, llr: torch.Tensor, w: torch.Tensor, tabs=None, pre_clamp=None) -> torch.Tensor:
    """Posterior L [B, n] of the unrolled weighted form (T = w.shape[0]) in torch FP64.
    pre_clamp: optional list that receives, per iteration t >= 1, the v->c sums A^(t+1)
    [B, E] before the clamp (for choosing test coordinates near or beyond it)."""
    chk_tab, var_tab, var_of_edge, E = tabs or _tables(code)
    B = llr.shape[0]
    T = w.shape[0]
    ct = torch.as_tensor(chk_tab)
    vt = torch.as_tensor(var_tab)
    voe = torch.as_tensor(var_of_edge)
    cmask = ct >= 0
    vmask = vt >= 0
    dc, dv = ct.shape[1], vt.shape[1]
    off_c = ~torch.eye(dc, dtype=torch.bool)
    off_v = ~torch.eye(dv, dtype=torch.bool)
    R_e = llr[:, voe]  # channel LLR seen on every edge [B, E]
    ones = torch.ones((), dtype=llr.dtype)
    zero = torch.zeros((), dtype=llr.dtype)
    WE = None
    for t in range(T):
        if t == 0:
            M = torch.clamp(R_e, -L_MAX, L_MAX)
        else:
            # sum over the other edges of each variable
            X = torch.where(vmask, WE[:, vt.clamp(min=0)], zero)  # [B, n, dv]
            excl = (X.unsqueeze(-2) * off_v).sum(-1)  # [B, n, dv]
            A = torch.zeros((B, E), dtype=llr.dtype)
            A[:, vt[vmask]] = (llr.unsqueeze(-1) + excl)[:, vmask]
            if pre_clamp is not None:
                pre_clamp.append(A.detach().clone())
            M = torch.clamp(A, -L_MAX, L_MAX)
        th = torch.where(cmask, torch.tanh(M[:, ct.clamp(min=0)] / 2.0), ones)  # [B, m, dc]
        P = torch.where(off_c, th.unsqueeze(-2), ones).prod(-1)  # product over the other edges
        Ecv = torch.zeros((B, E), dtype=llr.dtype)
        Ecv[:, ct[cmask]] = (2.0 * torch.atanh(P))[:, cmask]
        WE = w[t].unsqueeze(0) * Ecv
    if T == 0:
        return llr.clone()
    X = torch.where(vmask, WE[:, vt.clamp(min=0)], zero)
    return llr + X.sum(-1)


def loss_torch(L: torch.Tensor, cw: torch.Tensor) -> torch.Tensor:
    sp = torch.nn.functional.softplus
    return (cw * sp(L) + (1.0 - cw) * sp(-L)).mean()


def reference_grad(code, llr: np.ndarray, w: np.ndarray, cw: np.ndarray):
    """(loss, d loss / d llr [B, n], d loss / d w [T, E]) in FP64 via torch autograd."""
    lt = torch.tensor(np.asarray(llr, dtype=np.float64), requires_grad=True)
    wt = torch.tensor(np.asarray(w, dtype=np.float64), requires_grad=True)
    ct = torch.tensor(np.asarray(cw, dtype=np.float64))
    loss = loss_torch(forward_torch(code, lt, wt), ct)
    loss.backward()
    return float(loss.detach()), lt.grad.detach().numpy().copy(), wt.grad.detach().numpy().copy()


def loss_c(code, llr, w, cw) -> float:
    return bce_loss(unrolled(code, llr, w), cw)


def fd_grad(code, llr, w, cw, coords_w=(), coords_llr=(), rel_h: float = 1e-6):
    """Central differences of the C FP64 forward at the given (t, e) and (b, v) coordinates."""
    llr = np.array(llr, dtype=np.float64)
    w = np.array(w, dtype=np.float64)
    gw, gl = [], []
    for (t, e) in coords_w:
        x = w[t, e]
        h = rel_h * max(1.0, abs(x))
        w[t, e] = x + h
        fp = loss_c(code, llr, w, cw)
        w[t, e] = x - h
        fm = loss_c(code, llr, w, cw)
        w[t, e] = x
        gw.append((fp - fm) / (2 * h))
    for (b, v) in coords_llr:
        x = llr[b, v]
        h = rel_h * max(1.0, abs(x))
        llr[b, v] = x + h
        fp = loss_c(code, llr, w, cw)
        llr[b, v] = x - h
        fm = loss_c(code, llr, w, cw)
        llr[b, v] = x
        gl.append((fp - fm) / (2 * h))
    return np.array(gw), np.array(gl)
