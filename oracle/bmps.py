"""Boundary-MPS contraction of the single-layer network (Method section and
the Heisenberg benchmark, where the network rho_theta(S) is contracted with
boundary MPS of bond dimension D_c, written chi here).

The paper names the method and D_c but gives no algorithm.  Reading taken
(two-sweep SVD compression):

  * top[-1], bot[L1] are trivial (every leg of dimension 1);
  * top[r] = C_chi( top[r-1] o M_r ),  bot[r] = C_chi( M_r o bot[r+1] ),
    where "o" absorbs the row of slices M_r = (T_{r,c}^{S_{r,c}})_c into the
    boundary (bond dimensions multiply);
  * C_chi(A_0..A_{L-1}) with A_c[a, p, b]:
      1. left-to-right thin QR: A_c -> Q, A_{c+1} <- R A_{c+1};
      2. right-to-left SVD: A_c = U S V^T (as a x (p b)); keep
         k = min(chi, len(S)) values; A_c <- V^T[:k],
         A_{c-1} <- A_{c-1} U[:, :k] S[:k];
      3. n = ||A_0||_F, A_0 <- A_0 / n, log-scale += log n.
  * strip amplitudes: rho_r(S) = <top[r-1] | M_r | bot[r+1]>,
    rho_{r,r+1}(S) = <top[r-1] | M_r M_{r+1} | bot[r+2]>, both exact
    contractions of three (four) layers.

A Boundary is (list of tensors, log-scale); the amplitude of a strip is
exp(ls_top + ls_bot) * (contraction of the normalised tensors).
"""
from __future__ import annotations

import math

import numpy as np


def trivial(L2):
    """Boundary with every leg of dimension 1 (above row 0 / below row L1-1)."""
    return [np.ones((1, 1, 1)) for _ in range(L2)], 0.0


def absorb_top(A, W):
    """B_c[(a,l), d, (b,r)] = sum_u A_c[a,u,b] W_c[l,u,r,d]."""
    out = []
    for Ac, Wc in zip(A, W):
        a, _, b = Ac.shape
        l, _, r, d = Wc.shape
        out.append(np.einsum("aub,lurd->aldbr", Ac, Wc).reshape(a * l, d, b * r))
    return out


def absorb_bot(A, W):
    """B_c[(a,l), u, (b,r)] = sum_d A_c[a,d,b] W_c[l,u,r,d]."""
    out = []
    for Ac, Wc in zip(A, W):
        a, _, b = Ac.shape
        l, u, r, _ = Wc.shape
        out.append(np.einsum("adb,lurd->alubr", Ac, Wc).reshape(a * l, u, b * r))
    return out


def compress(A, chi):
    """C_chi of an open MPS; returns (tensors, log n).  log n = -inf when the
    MPS is identically zero."""
    A = [np.array(x, dtype=np.float64, copy=True) for x in A]
    L = len(A)
    for c in range(L - 1):
        a, p, b = A[c].shape
        Q, R = np.linalg.qr(A[c].reshape(a * p, b), mode="reduced")
        A[c] = Q.reshape(a, p, Q.shape[1])
        A[c + 1] = np.tensordot(R, A[c + 1], axes=(1, 0))
    for c in range(L - 1, 0, -1):
        a, p, b = A[c].shape
        U, s, Vt = np.linalg.svd(A[c].reshape(a, p * b), full_matrices=False)
        k = min(chi, len(s))
        A[c] = Vt[:k].reshape(k, p, b)
        A[c - 1] = np.tensordot(A[c - 1], U[:, :k] * s[:k], axes=(2, 0))
    n = float(np.linalg.norm(A[0]))
    if n == 0.0:
        return A, -math.inf
    A[0] = A[0] / n
    return A, math.log(n)


def bond_dims_after(shapes, chi):
    """Static bond dimensions produced by C_chi for given input shapes
    (a_c, p_c, b_c): they depend only on the shapes, never on the values."""
    L = len(shapes)
    a = [s[0] for s in shapes]
    p = [s[1] for s in shapes]
    b = [s[2] for s in shapes]
    for c in range(L - 1):
        k = min(a[c] * p[c], b[c])
        b[c] = k
        a[c + 1] = k
    for c in range(L - 1, 0, -1):
        k = min(chi, a[c], p[c] * b[c])
        a[c] = k
        b[c - 1] = k
    return [(a[c], p[c], b[c]) for c in range(L)]


def top_boundaries(lat, theta, config, chi):
    """[top[-1], top[0], ..., top[L1-1]] (index r+1)."""
    tops = [trivial(lat.L2)]
    for r in range(lat.L1):
        A, ls = tops[-1]
        B = absorb_top(A, lat.row_slices(theta, config, r))
        Ac, dl = compress(B, chi)
        tops.append((Ac, ls + dl))
    return tops


def bot_boundaries(lat, theta, config, chi):
    """[bot[0], ..., bot[L1-1], bot[L1]] (index r)."""
    bots = [None] * (lat.L1 + 1)
    bots[lat.L1] = trivial(lat.L2)
    for r in range(lat.L1 - 1, -1, -1):
        A, ls = bots[r + 1]
        B = absorb_bot(A, lat.row_slices(theta, config, r))
        Ac, dl = compress(B, chi)
        bots[r] = (Ac, ls + dl)
    return bots


def step1(E, Tc, Wc, Bc):
    """One column of a one-row strip: E[x,l,y] T[x,u,a] W[l,u,r,d] B[y,d,b]
    -> E'[a,r,b] (pairwise contractions, in this order)."""
    X = np.tensordot(E, Tc, axes=([0], [0]))            # [l, y, u, a]
    X = np.tensordot(X, Wc, axes=([0, 2], [0, 1]))      # [y, a, r, d]
    return np.tensordot(X, Bc, axes=([0, 3], [0, 1]))   # [a, r, b]


def step1_right(R, Tc, Wc, Bc):
    """Mirror of step1 from the right: R[a,r,b] -> R'[x,l,y]."""
    Y = np.tensordot(Bc, R, axes=([2], [2]))            # [y, d, a, r]
    Y = np.tensordot(Wc, Y, axes=([2, 3], [3, 1]))      # [l, u, y, a]
    return np.tensordot(Tc, Y, axes=([1, 2], [1, 3]))   # [x, l, y]


def step2(E, Tc, W1c, W2c, Bc):
    """One column of a two-row strip: E[x,l,m,y] T[x,u,a] W1[l,u,r,d]
    W2[m,d,s,e] B[y,e,b] -> E'[a,r,s,b]."""
    X = np.tensordot(E, Tc, axes=([0], [0]))            # [l, m, y, u, a]
    X = np.tensordot(X, W1c, axes=([0, 3], [0, 1]))     # [m, y, a, r, d]
    X = np.tensordot(X, W2c, axes=([0, 4], [0, 1]))     # [y, a, r, s, e]
    return np.tensordot(X, Bc, axes=([0, 4], [0, 1]))   # [a, r, s, b]


def strip1(top, W, bot):
    """<top | row | bot>: contraction of three layers, no truncation.
    top[c][a,u,a'], W[c][l,u,r,d], bot[c][b,d,b']."""
    E = np.ones((1, 1, 1))                      # [a, l, b]
    for Tc, Wc, Bc in zip(top, W, bot):
        E = step1(E, Tc, Wc, Bc)
    return float(E.reshape(()))


def strip2(top, W1, W2, bot):
    """<top | row r | row r+1 | bot>: four layers, no truncation."""
    E = np.ones((1, 1, 1, 1))                   # [a, l1, l2, b]
    for Tc, W1c, W2c, Bc in zip(top, W1, W2, bot):
        E = step2(E, Tc, W1c, W2c, Bc)
    return float(E.reshape(()))


def strip1_env(top, W, bot, c):
    """d <top|row|bot> / d W[c]: the environment of site c in a one-row strip,
    an array [l, u, r, d] (the strip is linear in W[c])."""
    L = np.ones((1, 1, 1))
    for j in range(c):
        L = step1(L, top[j], W[j], bot[j])
    R = np.ones((1, 1, 1))
    for j in range(len(W) - 1, c, -1):
        R = step1_right(R, top[j], W[j], bot[j])
    Z = np.tensordot(L, top[c], axes=([0], [0]))          # [l, y, u, a]
    Z = np.tensordot(Z, bot[c], axes=([1], [0]))          # [l, u, a, d, b]
    Z = np.tensordot(Z, R, axes=([2, 4], [0, 2]))         # [l, u, d, r]
    return Z.transpose(0, 1, 3, 2)
