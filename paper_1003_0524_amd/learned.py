"""Learned V^x extrapolator between exact evaluations (outer-iteration driver).

The paper keeps V^x fixed while the inner density iterations run and
recomputes it per outer step (Sec. IV, nested self-consistency). Because V^x
is linear in the density matrix P for fixed product-basis projections, the
change dV(k) caused by a change dP can be learned from the exact evaluations
the outer loop performs anyway. This module is the control flow of that
scheme; every arithmetic step runs in the library's kernels through the C ABI
(encoding: ``exchange_nn_features`` / ``exchange_nn_project``; network:
``exchange_nn_train`` / ``exchange_nn_predict``; prediction:
``exchange_nn_expand``; judge: ``exchange_eigh`` and the exact path
``exchange_matrix_all``). PyTorch holds device memory.

Schedule per outer iteration t = 1..n_iter (``run_outer``):
  * exact when t <= n_train, when t is a multiple of ``judge_every``, or while a
    failed judgement is pending; otherwise predicted;
  * exact iterations up to n_train give training pairs (dP, dV) between
    consecutive exact iterations; the network is trained after iteration n_train;
  * a prediction is V_anchor + |dP| * B dec(net(x)) B^H with the anchor the
    latest exact iteration and B the eigenvectors of the latest judged (or the
    last training) iteration for its n_blk most negative eigenvalues; when B
    changes, the stored pairs are projected onto the new B and the network is
    fine-tuned;
  * at judged iterations the prediction is compared with the exact result on every
    eigenvalue of every k (normalised by rho_max): the prediction changes V only
    inside span B, so the other n_b - n_blk eigenvalues keep the anchor's values and
    are judged too; above tau the scheme falls back to the exact path until a later
    judgement passes; the new exact pair is added to the training set and the
    network fine-tuned. The error on the n_blk most negative eigenvalues alone (the
    part the network predicts) is recorded beside it.
The stale-V scheme of the paper (prediction = anchor) is judged beside it.
"""
from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np


@dataclasses.dataclass
class Record:
    t: int
    exact: bool                    # the exact path ran
    used: str                      # "exact" or "predicted"
    judged: bool = False
    err_pred: Optional[float] = None           # every eigenvalue (decides acceptance)
    err_stale: Optional[float] = None
    err_ridge: Optional[float] = None
    err_pred_block: Optional[float] = None     # the n_blk most negative eigenvalues only
    err_stale_block: Optional[float] = None
    err_ridge_block: Optional[float] = None
    accepted: Optional[bool] = None
    train_loss: Optional[float] = None
    dp_norm: Optional[float] = None


class Extrapolator:
    """Network, encoding and basis of the learned dP -> dV map for one exchange context."""

    def __init__(self, ex, m: int = 64, n_blk: int = 8, hidden: int = 256, seed: int = 1,
                 sketch_seed: int = 0x5EED5EED, lr: float = 1e-3, epochs: int = 2000,
                 epochs_ft: int = 500, ridge_lambda: float = 1e-6):
        self.ex = ex
        self.t = ex._torch
        self.m, self.n_blk = int(m), int(n_blk)
        self.n_k = ex.n_k
        self.sketch_seed = sketch_seed
        self.lr, self.epochs, self.epochs_ft = lr, epochs, epochs_ft
        self.ridge_lambda = ridge_lambda
        # one sample per (dP, dV) pair: the sketch of dP in, the n_blk x n_blk blocks
        # of every k out (the k dependence of the linear response sits in the output layer)
        self.in_dim = self.m
        self.out_dim = self.n_k * self.n_blk * self.n_blk
        ex.nn_init(self.in_dim, hidden, self.out_dim, seed)
        self.Z = None                   # packed eigenvectors of the anchor (output basis)
        self.pairs = []                 # (V_new, V_old, |dP|) of every training pair (device copies)
        self.X: List[np.ndarray] = []   # training features (rows)
        self.Y: List[np.ndarray] = []   # training targets in the current basis (unscaled)
        self.y_scale = 1.0

    # -- encoding ------------------------------------------------------------
    def set_basis(self, V: Sequence) -> None:
        """Basis of the output encoding: eigenvectors of V (the anchor); the stored
        pairs are projected again onto it."""
        _, self.Z = self.ex.eigh(V)
        self.Y = [self.ex.nn_project(vn, vo, self.Z, self.n_blk, 1.0 / nrm).cpu().numpy().reshape(1, -1)
                  for (vn, vo, nrm) in self.pairs]

    def features(self, P_new, P_old) -> Tuple[np.ndarray, float]:
        """Feature row [1, m] (host float32) and |P_new - P_old|."""
        x, nrm = self.ex.nn_features(P_new, P_old, self.m, self.sketch_seed)
        return x.cpu().numpy().reshape(1, self.m), float(nrm.item())

    def add_pair(self, P_new, P_old, V_new, V_old) -> None:
        rows, nrm = self.features(P_new, P_old)
        if nrm == 0.0:
            return
        self.pairs.append(([v.clone() for v in V_new], [v.clone() for v in V_old], nrm))
        self.X.append(rows)
        if self.Z is not None:
            self.Y.append(self.ex.nn_project(V_new, V_old, self.Z, self.n_blk, 1.0 / nrm).cpu().numpy()
                          .reshape(1, -1))

    # -- network -------------------------------------------------------------
    def train(self, epochs: int) -> float:
        X = np.ascontiguousarray(np.concatenate(self.X))
        Y = np.concatenate(self.Y)
        self.y_scale = float(np.sqrt(np.mean(Y.astype(np.float64) ** 2))) or 1.0
        Ys = np.ascontiguousarray((Y / self.y_scale).astype(np.float32))
        return self.ex.nn_train(X, Ys, epochs, self.lr)

    def predict(self, P, P_anchor, V_anchor, outs, y_override: Optional[np.ndarray] = None):
        """V_anchor + |dP| B dec(y) B^H into outs (y from the network unless overridden)."""
        rows, nrm = self.features(P, P_anchor)
        if y_override is None:
            y = self.ex.nn_predict(self.t.from_numpy(rows).to(self.Z.device))
        else:
            y = self.t.from_numpy(np.ascontiguousarray(y_override, dtype=np.float32)).to(self.Z.device)
        y = y.reshape(self.n_k, self.n_blk * self.n_blk).contiguous()
        self.ex.nn_expand(V_anchor, self.Z, self.n_blk, y, nrm * self.y_scale, outs)
        return rows, nrm

    # -- comparison baseline (reported only, never used as the prediction) ------
    def ridge_y(self, rows: np.ndarray) -> np.ndarray:
        X = np.concatenate(self.X).astype(np.float64)
        Y = np.concatenate(self.Y).astype(np.float64) / self.y_scale
        Xa = np.hstack([X, np.ones((X.shape[0], 1))])
        W = np.linalg.solve(Xa.T @ Xa + self.ridge_lambda * np.eye(Xa.shape[1]), Xa.T @ Y)
        return np.hstack([rows, np.ones((rows.shape[0], 1))]) @ W

    # -- judge -----------------------------------------------------------------
    def spectrum(self, V: Sequence) -> List[np.ndarray]:
        """Ascending eigenvalues of V(k) for every k."""
        w, _ = self.ex.eigh(V)
        w = w.cpu().numpy()
        out, o = [], 0
        for nb in self.ex.n_bands:
            out.append(w[o:o + nb])
            o += nb
        return out

    def lowest(self, V: Sequence) -> np.ndarray:
        return np.array([w[:self.n_blk] for w in self.spectrum(V)])

    def judge(self, V_pred: Sequence, lam_exact: Sequence, rho_max: float) -> Tuple[float, float]:
        """(max over k and every eigenvalue, max over k and the n_blk lowest) of
        |lambda_pred - lambda_exact| / rho_max."""
        lam = self.spectrum(V_pred)
        full = max(float(np.max(np.abs(a - b))) for a, b in zip(lam, lam_exact))
        blk = max(float(np.max(np.abs(a[:self.n_blk] - b[:self.n_blk]))) for a, b in zip(lam, lam_exact))
        return full / rho_max, blk / rho_max


def _vec(ex, tensors):
    return [o.view(nb, nb).T for o, nb in zip(tensors, ex.n_bands)]


def run_outer(ex, feed: Callable[[int], Tuple[Sequence, object]], n_iter: int = 30, n_train: int = 10,
              judge_every: int = 5, tau: float = 1e-4, rho_max: Optional[float] = None, xp: Optional[Extrapolator] = None,
              ridge: bool = True, on_iter: Optional[Callable[[Record], None]] = None):
    """Run the outer-iteration schedule. ``feed(t)`` returns (M_t per k on the device,
    P_t as a float64/complex128 device vector). Returns (records, extrapolator, V of the
    last iteration as per-k column-major device buffers). ``rho_max`` (default: the
    largest |eigenvalue| of the first exact V^x) normalises the judged errors."""
    t_ = ex._torch
    dev = t_.device("cuda", ex.device)
    xp = xp or Extrapolator(ex)

    def buffers():
        return [t_.empty(nb * nb, dtype=t_.complex128, device=dev) for nb in ex.n_bands]

    V_anchor, V_prev, V_cur, V_tmp = buffers(), buffers(), buffers(), buffers()
    P_anchor = P_prev = None
    records: List[Record] = []
    fallback = False
    for t in range(1, n_iter + 1):
        M, P = feed(t)
        judged = t > n_train and t % judge_every == 0
        exact = t <= n_train or judged or fallback
        rec = Record(t=t, exact=exact, used="exact" if exact else "predicted", judged=judged)
        if exact:
            ex.matrix_all(M, V_cur)
        if t == 1:
            if rho_max is None:
                # the errors are reported on the scale where the largest |eigenvalue| of V^x is 1 Ha
                w, _ = ex.eigh(V_cur)
                rho_max = float(w.abs().max().item())
        if 1 < t <= n_train:
            xp.add_pair(P, P_prev, V_cur, V_prev)
        if t == n_train:
            xp.set_basis(V_cur)
            rec.train_loss = xp.train(xp.epochs)
        if t > n_train:
            if judged or not exact:
                rows, nrm = xp.predict(P, P_anchor, V_anchor, V_tmp)
                rec.dp_norm = nrm
            if judged:
                lam = xp.spectrum(V_cur)
                rec.err_pred, rec.err_pred_block = xp.judge(V_tmp, lam, rho_max)
                rec.err_stale, rec.err_stale_block = xp.judge(V_anchor, lam, rho_max)
                if ridge and xp.X:
                    xp.predict(P, P_anchor, V_anchor, V_tmp, y_override=xp.ridge_y(rows))
                    rec.err_ridge, rec.err_ridge_block = xp.judge(V_tmp, lam, rho_max)
                rec.accepted = rec.err_pred < tau
                fallback = not rec.accepted
                xp.add_pair(P, P_anchor, V_cur, V_anchor)
                xp.set_basis(V_cur)
                rec.train_loss = xp.train(xp.epochs_ft)
            elif not exact:
                for a, b in zip(V_cur, V_tmp):
                    a.copy_(b)
            else:
                xp.add_pair(P, P_anchor, V_cur, V_anchor)     # fallback iteration: one more exact pair
        if exact:
            for a, b in zip(V_anchor, V_cur):
                a.copy_(b)
            P_anchor = P
        for a, b in zip(V_prev, V_cur):
            a.copy_(b)
        P_prev = P
        records.append(rec)
        if on_iter:
            on_iter(rec)
    return records, xp, _vec(ex, V_cur)
