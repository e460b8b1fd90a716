"""Learned interpolation (oracle): features, targets, network, loss, Adam.

The paper has no learned component; this follows the build's reading:

* sample = an F point i of level 0 with a non-empty strong C set C_i;
* features (64): the same-component couplings a_ij / a_ii of row i placed in
  the 3x3x3 lattice box around node(i) (27 slots, slot = (dx+1) + 3(dy+1) +
  9(dz+1)), 27 flags for "j is in C_i", log10(kappa)/6 and two material
  constants, the one-hot component, zero padding;
* network 64 -> 64 -> 64 -> 27 (padded to 32), ReLU on the hidden layers,
  weights and activations rounded to bfloat16, accumulation in fp32;
* output: a correction added to the classical weights w_ij on the slots of
  C_i (masked); a zero last layer reproduces classical interpolation;
* target: the local ideal interpolation.  With F_loc = {i} and the F points
  of i's component among the columns of row i, solve
  A[F_loc, F_loc] X = -A[F_loc, C_i]; the row of X belonging to i is w*_i;
* loss: masked mean squared error of (w_classical + correction - w*);
* optimiser: Adam (Kingma & Ba 2015) on fp32 master weights.

The network is evaluated here in fp64 on operands rounded to bfloat16 the
same way as on the GPU (fp64 -> fp32 -> bf16 round-to-nearest-even).
"""
from __future__ import annotations

import numpy as np

NIN, NH, NOUT, NOUTP = 64, 64, 27, 32
# flat parameter layout: W1 [64x64] (in x out), b1 [64], W2 [64x64], b2 [64], W3 [64x32], b3 [32]
SHAPES = [("W1", (NIN, NH)), ("b1", (NH,)), ("W2", (NH, NH)), ("b2", (NH,)), ("W3", (NH, NOUTP)), ("b3", (NOUTP,))]
NPARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(flat):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(flat[o:o + k], dtype=np.float64).reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], np.float32).ravel() for name, _ in SHAPES])


def init_weights(seed=0):
    """He-normal hidden layers, zero last layer (network == classical)."""
    r = np.random.default_rng(seed)
    w = {"W1": r.normal(0, np.sqrt(2.0 / NIN), (NIN, NH)), "b1": np.zeros(NH),
         "W2": r.normal(0, np.sqrt(2.0 / NH), (NH, NH)), "b2": np.zeros(NH),
         "W3": np.zeros((NH, NOUTP)), "b3": np.zeros(NOUTP)}
    return pack(w)


def bf16(x):
    """Round to bfloat16 (nearest, ties to even) through fp32; returns fp64 values."""
    f = np.asarray(x, dtype=np.float64).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def slot_of(off):
    return int((off[0] + 1) + 3 * (off[1] + 1) + 9 * (off[2] + 1))


def material_features(materials):
    m = materials[0]
    second = m["c01"] if int(m["model"]) == 0 else m["k1"]
    return np.array([np.log10(m["kappa"]) / 6.0, m["c10"], second])


def samples(A, comp, state, S_ptr, S_idx, P, lattice, matfeat):
    """Features X [M,64], mask [M,27], base weights [M,27] and the row
    indices of the samples, in ascending row order.  Features: the stencil
    a_ij / a_ii of the same-component neighbours in the 3x3x3 lattice box;
    mask and base weights: the entries of the row of P (classical or
    extended+i) whose C point lies in the box."""
    n = A.shape[0]
    rows, X, mask, wcl = [], [], [], []
    c2f = np.flatnonzero(state == 1)
    for i in range(n):
        if state[i] != -1 or P.indptr[i + 1] == P.indptr[i]:
            continue
        node, c = i // 3, comp[i]
        lo, hi = A.indptr[i], A.indptr[i + 1]
        cols, vals = A.indices[lo:hi], A.data[lo:hi]
        aii = vals[cols == i][0]
        x = np.zeros(NIN)
        mk = np.zeros(NOUT)
        w = np.zeros(NOUT)
        for j, a in zip(cols, vals):
            if comp[j] != c:
                continue
            off = lattice[j // 3] - lattice[node]
            if np.abs(off).max() > 1:
                continue
            x[slot_of(off)] = np.float32(a / aii)
        for q in range(P.indptr[i], P.indptr[i + 1]):
            off = lattice[c2f[P.indices[q]] // 3] - lattice[node]
            if np.abs(off).max() > 1:
                continue
            s = slot_of(off)
            x[27 + s] = 1.0
            mk[s] = 1.0
            w[s] = P.data[q]
        x[54:57] = np.float32(matfeat)
        x[57 + c] = 1.0
        rows.append(i)
        X.append(x)
        mask.append(mk)
        wcl.append(w)
    return np.array(rows, np.int64), np.array(X), np.array(mask), np.array(wcl)


def ideal_target(A, comp, state, S_ptr, S_idx, lattice, i, classical_sum=None, P=None):
    """w*_i on the 27 slots (zero outside C_i).

    C_i: the strong C neighbours of i, or, with P given, the C points of the
    row of P (which may reach beyond the lattice box).  F_loc: i and the
    same-component F points of row i.  w*_i solves A_FF X = -A_FC on F_loc x
    C_i; only C points inside the box get a slot.  With classical_sum given,
    the in-box part of w*_i is rescaled to that sum: the local system drops
    every coupling outside F_loc, so its raw solution does not reproduce
    constants; the base weights do (for zero row sums), and an
    interpolation that loses them slows the V-cycle down."""
    lo, hi = A.indptr[i], A.indptr[i + 1]
    cols = A.indices[lo:hi]
    if P is None:
        S_set = set(S_idx[S_ptr[i]:S_ptr[i + 1]].tolist())
        Ci = [int(j) for j in cols if j in S_set and state[j] == 1]
    else:
        c2f = np.flatnonzero(state == 1)
        Ci = [int(c2f[q]) for q in P.indices[P.indptr[i]:P.indptr[i + 1]]]
    Floc = [int(j) for j in cols if comp[j] == comp[i] and (j == i or state[j] == -1)]
    Ad = A[Floc][:, Floc].toarray()
    Ac = A[Floc][:, Ci].toarray()
    Xs = np.linalg.solve(Ad, -Ac)
    wi = Xs[Floc.index(i)]
    inbox = [bool(np.abs(lattice[j // 3] - lattice[i // 3]).max() <= 1) for j in Ci]
    if classical_sum is not None:
        s = 0.0
        for w, ib in zip(wi, inbox):
            if ib:
                s += w
        if abs(s) > 1e-12:
            wi = wi * (classical_sum / s)
    out = np.zeros(NOUT)
    for j, w, ib in zip(Ci, wi, inbox):
        if ib:
            out[slot_of(lattice[j // 3] - lattice[i // 3])] = w
    return out


def forward(X, flat, rounding=True):
    """Returns (out [M,32], h1, h2, x) with bf16-rounded operands
    (rounding=False evaluates the same network in plain fp64)."""
    p = unpack(flat)
    rd = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    x = rd(X)
    h1 = rd(np.maximum(x @ rd(p["W1"]) + p["b1"], 0.0))
    h2 = rd(np.maximum(h1 @ rd(p["W2"]) + p["b2"], 0.0))
    out = h2 @ rd(p["W3"]) + p["b3"]
    return out, h1, h2, x


def loss_and_grad(X, mask, wcl, wstar, flat, acts=None, rounding=True):
    """Masked MSE and its gradient w.r.t. the flat parameters.

    acts = (h1, h2, x) lets a caller supply the bf16 activations of another
    forward evaluation so that the backward pass sees identical operands."""
    p = unpack(flat)
    rd = bf16 if rounding else (lambda a: np.asarray(a, np.float64))
    out, h1, h2, x = forward(X, flat, rounding)
    if acts is not None:
        h1, h2, x = acts
        out = h2 @ rd(p["W3"]) + p["b3"]
    cnt = max(mask.sum(), 1.0)
    r = (wcl + out[:, :NOUT] - wstar) * mask
    loss = float((r * r).sum() / cnt)
    dout = np.zeros_like(out)
    dout[:, :NOUT] = 2.0 * r / cnt
    g = {"W3": h2.T @ dout, "b3": dout.sum(0)}
    dh2 = (dout @ rd(p["W3"]).T) * (h2 > 0)
    g["W2"], g["b2"] = h1.T @ dh2, dh2.sum(0)
    dh1 = (dh2 @ rd(p["W2"]).T) * (h1 > 0)
    g["W1"], g["b1"] = x.T @ dh1, dh1.sum(0)
    return loss, np.concatenate([g[name].ravel() for name, _ in SHAPES])


def adam_step(flat, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    m = b1 * m + (1 - b1) * grad
    v = b2 * v + (1 - b2) * grad * grad
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return flat - lr * mh / (np.sqrt(vh) + eps), m, v
