"""Learned first guess for the self-consistent Hamiltonian loop (oracle; test
infrastructure only).

Algorithm 1 starts each step's self-consistency loop from the linear
extrapolation H_1 = 2 H_0 - H_-1.  With fixed orbitals H is affine in the
Hartree-exchange potential, so that guess is the potential 2 V_j - V_(j-1), and
its error is the second difference D_j = V_(j+1) - 2 V_j + V_(j-1) of the
converged potentials.  The learned predictor adds h^3 Psi^T diag(P r) Psi,
where r is a network's estimate of R D_j on a coarse 16^3 grid, R the
restriction and P the prolongation below.  The loop still iterates to the same
fixed point: the network only changes where it starts (predictor-independence
is the invariant the tests check).

Definitions used by both the oracle and, independently written, the kernels:
  * R: average over the n/16 x n/16 x n/16 block of fine points of each coarse
    cell (grid edges divisible by 16).
  * P: periodic trilinear interpolation from coarse cell centres, coarse cell
    c along an axis sits at fine coordinate (c + 1/2) b - 1/2, b = n / 16.
  * moments of a density change d (9 numbers): h^3 sum d q_a and
    h^3 sum d q_a q_b (a <= b), q the centred sawtooth coordinates.
  * network: x (8264) -> tanh(W1 x + b1) (256) -> tanh(W2 . + b2) (256) ->
    W3 . + b3 (4096), inputs and outputs standardised by stored mean/scale.
  * loss: mean over batch and outputs of (y - t)^2 / 2.
"""

import numpy as np

NC = 16  # coarse grid edge
N_IN = 8 * 9 + 2 * NC ** 3  # 8 past moment vectors + two coarse density snapshots
N_H = 256
N_OUT = NC ** 3


def restrict(f: np.ndarray, n) -> np.ndarray:
    """Block average of a fine field [nz, ny, nx] (flattened ok) onto 16^3."""
    nx, ny, nz = n
    f = f.reshape(nz, ny, nx)
    bz, by, bx = nz // NC, ny // NC, nx // NC
    return f.reshape(NC, bz, NC, by, NC, bx).mean(axis=(1, 3, 5))


def _interp_weights(n_fine: int):
    """For each fine index: (c0, c1, w1) with value = (1-w1) g[c0] + w1 g[c1]."""
    b = n_fine // NC
    x = (np.arange(n_fine) + 0.5) / b - 0.5  # position in coarse-centre units
    c0 = np.floor(x).astype(int)
    w1 = x - c0
    return c0 % NC, (c0 + 1) % NC, w1


def prolong(g: np.ndarray, n) -> np.ndarray:
    """Periodic trilinear interpolation of a coarse field [16,16,16] to [nz, ny, nx]."""
    nx, ny, nz = n
    out = g.reshape(NC, NC, NC)
    for axis, nf in ((0, nz), (1, ny), (2, nx)):
        c0, c1, w1 = _interp_weights(nf)
        a = np.take(out, c0, axis=axis)
        b = np.take(out, c1, axis=axis)
        shape = [1, 1, 1]
        shape[axis] = nf
        w = w1.reshape(shape)
        out = (1 - w) * a + w * b
    return out


def moments(d: np.ndarray, qs, h: float) -> np.ndarray:
    """9 moments of a density change: dipole (3) and second moments (6)."""
    dv = h ** 3
    m = [dv * np.sum(d * q) for q in qs]
    for a in range(3):
        for b in range(a, 3):
            m.append(dv * np.sum(d * qs[a] * qs[b]))
    return np.array(m)


def features(mom_hist, drho_t, drho_tm1, n) -> np.ndarray:
    """Network input: 8 moment vectors (oldest first) + R(drho_t) + R(drho_(t-1))."""
    m = np.concatenate([np.asarray(v) for v in mom_hist[-8:]])
    return np.concatenate([m, restrict(drho_t, n).ravel(), restrict(drho_tm1, n).ravel()])


def init_params(seed: int = 0, n_in=N_IN, n_h=N_H, n_out=N_OUT):
    rng = np.random.default_rng(seed)
    return {
        "W1": rng.standard_normal((n_h, n_in)) / np.sqrt(n_in), "b1": np.zeros(n_h),
        "W2": rng.standard_normal((n_h, n_h)) / np.sqrt(n_h), "b2": np.zeros(n_h),
        "W3": rng.standard_normal((n_out, n_h)) * 0.01 / np.sqrt(n_h), "b3": np.zeros(n_out),
    }


def forward(p, X):
    """X [B, n_in] -> (Y [B, n_out], cache)."""
    z1 = X @ p["W1"].T + p["b1"]
    a1 = np.tanh(z1)
    z2 = a1 @ p["W2"].T + p["b2"]
    a2 = np.tanh(z2)
    Y = a2 @ p["W3"].T + p["b3"]
    return Y, (X, a1, a2)


def loss_and_grads(p, X, Tgt):
    """Mean-square loss sum((Y - T)^2) / (2 B n_out) and its gradients (backpropagation)."""
    Y, (X, a1, a2) = forward(p, X)
    B, n_out = Y.shape
    dY = (Y - Tgt) / (B * n_out)
    loss = 0.5 * np.sum((Y - Tgt) ** 2) / (B * n_out)
    g = {"W3": dY.T @ a2, "b3": dY.sum(0)}
    d2 = (dY @ p["W3"]) * (1 - a2 ** 2)
    g["W2"] = d2.T @ a1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1 - a1 ** 2)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    return loss, g


def adam(p, g, state, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (Kingma & Ba 2015) in place; state holds m, v, t."""
    state["t"] = state.get("t", 0) + 1
    t = state["t"]
    for k in p:
        m = state.setdefault("m_" + k, np.zeros_like(p[k]))
        v = state.setdefault("v_" + k, np.zeros_like(p[k]))
        m[...] = b1 * m + (1 - b1) * g[k]
        v[...] = b2 * v + (1 - b2) * g[k] ** 2
        mh = m / (1 - b1 ** t)
        vh = v / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)
