"""TEST INFRASTRUCTURE ONLY: the training loss of a se_e2_a model and its parameter gradient, in plain
PyTorch (FP64, CPU) with autograd as the differentiation primitive.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may use it.

What it computes (paper Sec. II.B, "Trainer"):
  * the model energy E(r; theta) = sum_i F_0(D^i) written out from Sec. II.A.1 and II.A.2: the
    switching function (eq. switch), environment rows R_j = s(r_j) (1, r_j / r_j), embedding nets
    G = N(s) with the layers of eq. NN, T = N_c^-1 G^T R, D = T T_<^T, fitting nets F_0;
  * forces F = -dE/dr (autograd with a graph, so that they can be differentiated again) and the
    virial Xi_ab = -sum_ij (dE/dr_ij)_a (r_ij)_b over the neighbour pairs;
  * the loss of eq. loss for one frame, L = p_E L_E + p_F L_F + p_Xi L_Xi with
    L_E = (E - E*)^2 / N, L_F = sum_k q_k |F_k - F*_k|^2 / (3N) (q_k = 1 unless given: the
    prefactor form L_F^p; q_k = 1/|F*_k|^2 gives the relative form L_F^r) and
    L_Xi = sum_ab (Xi - Xi*)_ab^2 / (9N);
  * dL/dtheta for every entry of the FP64 parameter blob (double backward through the forces);
  * the learning rate of eq. learning_rate and the prefactor schedule p(tau);
  * one Adam step (Kingma and Ba, the optimiser the paper names).

The neighbour list (which j are neighbours of i and the periodic image of each pair) is taken from
the C oracle's search (a discrete choice, not differentiated); r_ij itself is recomputed here from
the coordinates so that it carries the autograd graph.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import Oracle


def _layers(model: dict, params: torch.Tensor):
    """Views of every layer (W [nin][nout], b, w_hat) in the blob order: embedding nets, then one
    fitting net per type."""
    nt = model["ntypes"]
    nets = nt if model["type_one_side"] else nt * nt
    e = [1] + list(model["emb"])
    f = [model["emb"][-1] * model["axis"]] + list(model["fit"]) + [1]
    off = 0

    def take(nin, nout):
        nonlocal off
        W = params[off:off + nin * nout].view(nin, nout)
        off += nin * nout
        b = params[off:off + nout]
        off += nout
        wh = params[off:off + nout]
        off += nout
        return W, b, wh

    emb = [[take(e[k], e[k + 1]) for k in range(3)] for _ in range(nets)]
    fit = [[take(f[k], f[k + 1]) for k in range(4)] for _ in range(nt)]
    assert off == params.numel()
    return emb, fit


def _skip(x, nin, nout):
    if nout == nin:
        return x
    if nout == 2 * nin:
        return torch.cat([x, x], dim=-1)
    return 0.0


def _hidden(x, layer):
    W, b, wh = layer
    return wh * torch.tanh(x @ W + b) + _skip(x, W.shape[0], W.shape[1])


def _switch(r, rs, rc):
    """s(r) of eq. switch: 1/r below r_s, u(x)/r between, 0 from r_c on (u the quintic)."""
    x = ((r - rs) / (rc - rs)).clamp(0.0, 1.0)
    u = x ** 3 * (-6.0 * x ** 2 + 15.0 * x - 10.0) + 1.0
    return torch.where(r < rs, 1.0 / r, torch.where(r < rc, u / r, torch.zeros_like(r)))


def energy_graph(model: dict, params: torch.Tensor, coord: torch.Tensor, atype: np.ndarray, nl: np.ndarray,
                 shift: np.ndarray):
    """E (and E_i, r_ij) as torch functions of params and coord. nl [N][N_c] neighbour indices (-1
    padding), shift [N][N_c][3] the periodic image offset of each pair."""
    n, nc = nl.shape
    nt = model["ntypes"]
    emb, fit = _layers(model, params)
    M, A = model["emb"][-1], model["axis"]
    sel = model["sel"]
    off = np.concatenate([[0], np.cumsum(sel)])
    ii, slot = np.nonzero(nl >= 0)
    jj = nl[ii, slot]
    ti = atype[ii]
    tj = np.searchsorted(off, slot, side="right") - 1
    net = tj if model["type_one_side"] else ti * nt + tj
    ii_t, jj_t = torch.from_numpy(ii), torch.from_numpy(jj)
    rij = coord[jj_t] - coord[ii_t] + torch.from_numpy(shift[ii, slot])
    r = torch.linalg.norm(rij, dim=1)
    s = _switch(r, model["rcut_smth"], model["rcut"])
    R = torch.cat([s[:, None], (s / r)[:, None] * rij], dim=1)          # [P][4]
    G = torch.zeros(len(ii), M, dtype=torch.float64)
    for e_ in range(len(emb)):
        sel_p = torch.from_numpy(np.nonzero(net == e_)[0])
        if len(sel_p) == 0:
            continue
        h = s[sel_p, None]
        for layer in emb[e_]:
            h = _hidden(h, layer)
        G = G.index_copy(0, sel_p, h)
    # T_i = N_c^-1 sum_j G_j^T R_j  [N][M][4]
    T = torch.zeros(n, M, 4, dtype=torch.float64).index_add(0, ii_t, G[:, :, None] * R[:, None, :]) / nc
    D = torch.einsum("imk,ink->imn", T, T[:, :A, :]).reshape(n, M * A)
    Ei = torch.zeros(n, dtype=torch.float64)
    for t in range(nt):
        idx = torch.from_numpy(np.nonzero(atype == t)[0])
        if len(idx) == 0:
            continue
        h = D[idx]
        for layer in fit[t][:3]:
            h = _hidden(h, layer)
        W, b, wh = fit[t][3]
        Ei = Ei.index_copy(0, idx, (wh * (h @ W + b))[:, 0])
    return Ei.sum(), Ei, rij, ii, jj


class TrainOracle:
    """Loss and gradient of one frame for a se_e2_a model (dict) and its FP64 blob."""

    def __init__(self, model: dict, params: np.ndarray):
        assert model.get("descriptor", "se_e2_a") == "se_e2_a"
        self.model = dict(model)
        self.params = np.array(params, dtype=np.float64)
        self.c_oracle = Oracle(model, self.params)

    def _graph(self, coord, atype, box, params_t):
        nl, rij_np, _ = self.c_oracle.nlist(coord, atype, box)
        n = len(atype)
        ii, slot = np.nonzero(nl >= 0)
        shift = np.zeros(rij_np.shape)
        shift[ii, slot] = rij_np[ii, slot] - (coord[nl[ii, slot]] - coord[ii])
        coord_t = torch.tensor(coord, dtype=torch.float64, requires_grad=True)
        E, Ei, rij, _, _ = energy_graph(self.model, params_t, coord_t, np.asarray(atype), nl, shift)
        gc, gr = torch.autograd.grad(E, [coord_t, rij], create_graph=True)
        F = -gc
        Xi = -(gr[:, :, None] * rij[:, None, :]).sum(0)
        return E, Ei, F, Xi, n

    def predict(self, coord, atype, box):
        """E, F, Xi, E_i of the current parameters (plain values)."""
        params_t = torch.tensor(self.params, dtype=torch.float64)
        E, Ei, F, Xi, _ = self._graph(np.asarray(coord, dtype=np.float64), atype, box, params_t)
        return dict(energy=E.item(), force=F.detach().numpy(), virial=Xi.detach().numpy(),
                    atom_energy=Ei.detach().numpy())

    def loss_and_grad(self, coord, atype, box, e_label=None, f_label=None, v_label=None, pe=0.0, pf=0.0, pv=0.0,
                      atom_pref=None, grad=True):
        """(L, {"E": L_E, "F": L_F, "Xi": L_Xi}, dL/dtheta) of eq. loss for one frame. A term whose
        label is None is left out."""
        coord = np.asarray(coord, dtype=np.float64)
        params_t = torch.tensor(self.params, dtype=torch.float64, requires_grad=grad)
        E, Ei, F, Xi, n = self._graph(coord, atype, box, params_t)
        zero = torch.zeros((), dtype=torch.float64)
        LE = (E - float(e_label)) ** 2 / n if e_label is not None else zero
        if f_label is not None:
            q = torch.ones(n, dtype=torch.float64) if atom_pref is None else torch.tensor(atom_pref, dtype=torch.float64)
            LF = (q[:, None] * (F - torch.tensor(f_label, dtype=torch.float64)) ** 2).sum() / (3 * n)
        else:
            LF = zero
        LV = ((Xi - torch.tensor(np.asarray(v_label).reshape(3, 3), dtype=torch.float64)) ** 2).sum() / (9 * n) \
            if v_label is not None else zero
        L = pe * LE + pf * LF + pv * LV
        g = torch.autograd.grad(L, params_t)[0].numpy() if grad else None
        return L.item(), {"E": LE.item(), "F": LF.item(), "Xi": LV.item()}, g


def learning_rate(lr0: float, lr_stop: float, step: int, stop_steps: int, decay_steps: int) -> float:
    """eq. learning_rate: gamma(tau) = gamma0 r^floor(tau / s), r = (gamma_stop / gamma0)^(s / tau_stop)."""
    r = (lr_stop / lr0) ** (decay_steps / stop_steps)
    return lr0 * r ** (step // decay_steps)


def prefactor(p_start: float, p_limit: float, lr: float, lr0: float) -> float:
    """p(tau) = p_limit (1 - gamma/gamma0) + p_start gamma/gamma0."""
    return p_limit * (1.0 - lr / lr0) + p_start * lr / lr0


def adam_step(theta, grad, m, v, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba, Algorithm 1), step counted from 1: returns theta, m, v."""
    m = beta1 * m + (1.0 - beta1) * grad
    v = beta2 * v + (1.0 - beta2) * grad * grad
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v
