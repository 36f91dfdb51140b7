"""Per-element error bound of the GPU's float32 CDF-network gradient, derived
from the kernel's operation order (test infrastructure, CPU only).

Every quantity q of the forward and backward pass is carried as a pair
(|q|, e_q): its magnitude in float64 and a first-order bound on the error of
its float32 value, with u = 2^-24 and gamma_k = k u / (1 - k u) (Higham,
Accuracy and Stability of Numerical Algorithms, 2nd ed., Lemma 3.1 and
Sec. 4.2 for recursive summation):
  * a product a*b: e = |a| e_b + |b| e_a + u |a b|;
  * a sum of k terms added one after another: e = sum e_i + gamma_k sum |t_i|;
  * the ramp r(z) = min(max(z, 0), 1) is 1-Lipschitz: e_r(z) <= e_z;
  * its derivative r'(z) (0 or 1) is exact unless z lies within e_z of 0 or 1,
    where the GPU may take the other branch ("ambiguous").
The kernel sums each gradient entry over the 256 samples of a workgroup, in
order, then the workgroups' partials in order, so an entry's summation error
is at most (gamma_256 + gamma_nblk) sum_s |t_s|.  A sample with an ambiguous
derivative contributes its whole term magnitude to the bound of every entry
(the term may be present on one side and absent on the other).

grad_bound(p, x, y) returns the bound per parameter (1153 values), in the
parameter order of oracle.mlp.  float32_grad(p, x, y) emulates the kernel's
order in numpy float32 (separate multiply and add), for the CPU check that the
bound holds where the rounding is known.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp as M

U = 2.0 ** -24
BLOCK = 256


def gamma(k):
    return k * U / (1 - k * U)


def _ramp(z):
    return np.minimum(np.maximum(z, 0.0), 1.0)


def grad_bound(p, x, y):
    W1, b1, W2, b2, W3, b3 = M.unpack(np.asarray(p, np.float64))
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    m = x.shape[0]
    H = M.H
    # ---- forward: values and error bounds
    z1 = x[:, None] * W1[None, :] + b1[None, :]
    e_z1 = gamma(2) * (np.abs(x[:, None] * W1[None, :]) + np.abs(b1)[None, :])
    h1 = _ramp(z1)
    e_h1 = e_z1
    z2 = h1 @ W2.T + b2[None, :]
    a_z2 = np.abs(h1) @ np.abs(W2).T + np.abs(b2)[None, :]
    e_z2 = gamma(H + 1) * a_z2 + e_h1 @ np.abs(W2).T
    h2 = _ramp(z2)
    e_h2 = e_z2
    f = h2 @ W3 + b3
    e_f = gamma(H + 1) * (np.abs(h2) @ np.abs(W3) + abs(b3)) + e_h2 @ np.abs(W3)
    r = f - y
    e_r = e_f + U * np.abs(r)
    df = 2.0 * r / m
    e_df = 2.0 * e_r / m + U * np.abs(df)
    a_df = np.abs(df)
    # ambiguous derivative branches
    amb2 = (np.abs(z2) <= e_z2) | (np.abs(z2 - 1.0) <= e_z2)
    amb1 = (np.abs(z1) <= e_z1) | (np.abs(z1 - 1.0) <= e_z1)
    d2 = ((z2 > 0) & (z2 < 1)).astype(np.float64)
    d1 = ((z1 > 0) & (z1 < 1)).astype(np.float64)
    d2h = np.maximum(d2, amb2)            # derivative taken as 1 where ambiguous
    d1h = np.maximum(d1, amb1)
    # ---- backward: magnitudes (with ambiguous derivatives as 1) and errors
    a_dz2 = a_df[:, None] * np.abs(W3)[None, :] * d2h
    e_dz2 = (e_df[:, None] * np.abs(W3)[None, :] + U * a_dz2) * d2h
    a_s1 = a_dz2 @ np.abs(W2)                               # |sum_o dz2 W2| terms
    e_s1 = e_dz2 @ np.abs(W2) + gamma(H) * a_s1 + U * a_s1
    a_dz1 = a_s1 * d1h
    e_dz1 = e_s1 * d1h
    nblk = (m + BLOCK - 1) // BLOCK
    gs = gamma(BLOCK) + gamma(nblk)

    def entry(a_terms, e_terms):
        """Bound of sum_s t_s from per-sample |t_s| and term errors, [m, k]."""
        return e_terms.sum(axis=0) + gs * a_terms.sum(axis=0)

    ah2 = np.abs(h2)
    ah1 = np.abs(h1)
    ax = np.abs(x)
    # gW3[o] = sum_s df h2[s,o]
    bW3 = entry(a_df[:, None] * ah2, e_df[:, None] * ah2 + a_df[:, None] * e_h2
                + U * a_df[:, None] * ah2)
    bb3 = entry(a_df[:, None], e_df[:, None])[0]
    # gW2[o,i] = sum_s dz2[s,o] h1[s,i]; gb2[o] = sum_s dz2[s,o]
    a_w2 = a_dz2.T @ ah1                                    # [o, i] sums of |terms|
    e_w2 = e_dz2.T @ ah1 + a_dz2.T @ e_h1 + U * a_w2
    bW2 = e_w2 + gs * a_w2
    bb2 = entry(a_dz2, e_dz2)
    # gW1[i] = sum_s dz1[s,i] x_s; gb1[i] = sum_s dz1[s,i]
    bW1 = entry(a_dz1 * ax[:, None], e_dz1 * ax[:, None] + U * a_dz1 * ax[:, None])
    bb1 = entry(a_dz1, e_dz1)
    bound = M.pack(bW1, bb1, bW2, bb2, bW3, bb3)
    # samples with an ambiguous branch: their whole term magnitude, per entry
    amb = amb1.any(axis=1) | amb2.any(axis=1)
    if amb.any():
        s = amb
        ext = M.pack((a_dz1[s] * ax[s, None]).sum(axis=0), a_dz1[s].sum(axis=0),
                     a_dz2[s].T @ ah1[s], a_dz2[s].sum(axis=0),
                     (a_df[s, None] * ah2[s]).sum(axis=0), a_df[s].sum())
        bound = bound + 2.0 * ext
    return bound, int(amb.sum())


def float32_grad(p, x, y):
    """The kernel's gradient in numpy float32, in its order of operations."""
    f32 = np.float32
    W1, b1, W2, b2, W3, b3 = (np.asarray(a, f32) for a in M.unpack(np.asarray(p, np.float32)))
    b3 = f32(b3)
    x = np.asarray(x, f32)
    y = np.asarray(y, f32)
    m = x.shape[0]
    H = M.H
    z1 = x[:, None] * W1[None, :] + b1[None, :]
    h1 = np.minimum(np.maximum(z1, f32(0)), f32(1))
    z2 = np.repeat(b2[None, :], m, axis=0)
    for i in range(H):
        z2 = z2 + W2[None, :, i] * h1[:, i:i + 1]
    f = np.full(m, b3, f32)
    for o in range(H):
        f = f + W3[o] * np.minimum(np.maximum(z2[:, o], f32(0)), f32(1))
    r = f - y
    df = f32(2) * r / f32(m)
    h2 = np.minimum(np.maximum(z2, f32(0)), f32(1))
    d2 = ((z2 > 0) & (z2 < 1)).astype(f32)
    d1 = ((z1 > 0) & (z1 < 1)).astype(f32)
    dz2 = df[:, None] * W3[None, :] * d2
    s1 = np.zeros((m, H), f32)
    for o in range(H):
        s1 = s1 + dz2[:, o:o + 1] * W2[None, o, :]
    dz1 = s1 * d1

    def blocked(terms):
        """Sum over samples: in order inside 256-sample blocks, then blocks in order."""
        t = terms.reshape(m, -1)
        nblk = (m + BLOCK - 1) // BLOCK
        tot = np.zeros(t.shape[1], f32)
        for b in range(nblk):
            part = np.add.accumulate(t[b * BLOCK:(b + 1) * BLOCK], axis=0, dtype=f32)[-1]
            tot = tot + part
        return tot

    gW3 = blocked(df[:, None] * h2)
    gb3 = blocked(df[:, None])[0]
    gW2 = blocked((dz2[:, :, None] * h1[:, None, :]).reshape(m, -1)).reshape(H, H)
    gb2 = blocked(dz2)
    gW1 = blocked(dz1 * x[:, None])
    gb1 = blocked(dz1)
    return M.pack(gW1.astype(np.float64), gb1.astype(np.float64), gW2.astype(np.float64),
                  gb2.astype(np.float64), gW3.astype(np.float64), float(gb3))
