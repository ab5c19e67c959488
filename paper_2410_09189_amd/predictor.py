"""Training driver for the learned first guess (orchestration only).

Samples are recorded by the time step itself (rt_record: features x_j and the
realised coarse second difference of the Hartree-exchange potential), and the
network is trained on the GPU with the library's own kernels (rt_mlp_colstats
for standardisation, rt_mlp_loss_grad for forward + backpropagation,
rt_mlp_adam).  PyTorch only holds device memory.
"""

import numpy as np

from . import rt


def init_params(dims, seed=0):
    """Packed parameters (host float32): identity standardisation, scaled
    Gaussian weights, zero biases, small last layer."""
    n_in, n_h, n_out = dims
    rng = np.random.default_rng(seed)
    parts = [
        np.zeros(n_in), np.ones(n_in), np.zeros(n_out), np.ones(n_out),
        rng.standard_normal((n_h, n_in)) / np.sqrt(n_in), np.zeros(n_h),
        rng.standard_normal((n_h, n_h)) / np.sqrt(n_h), np.zeros(n_h),
        rng.standard_normal((n_out, n_h)) * 0.01 / np.sqrt(n_h), np.zeros(n_out),
    ]
    p = np.concatenate([a.ravel() for a in parts]).astype(np.float32)
    assert p.size == rt.rt_mlp_n_params(*dims)
    return p


def train_offset(dims):
    n_in, n_h, n_out = dims
    return 2 * n_in + 2 * n_out


def record(session_factory, n_steps, capacity):
    """Runs a session with recording on; returns device tensors (X, Y) of the rows written."""
    import torch

    n_in, _, n_out = rt.rt_mlp_dims()
    X = torch.empty((capacity, n_in), dtype=torch.float32, device="cuda")
    Y = torch.empty((capacity, n_out), dtype=torch.float32, device="cuda")
    ses = session_factory()
    rt.rt_record(ses.ctx, X.data_ptr(), Y.data_ptr(), capacity)
    rt.rt_step(ses.ctx, n_steps)
    n = rt.rt_record_count(ses.ctx)
    ses.close()
    return X[:n], Y[:n]


def train(X, Y, dims=None, epochs=40, batch=64, lr=1e-3, seed=0, floor_std=1e-6, log=None):
    """Fits the network to (X, Y) (device float32 tensors).  Returns (packed host
    params, per-epoch mean loss)."""
    import torch

    dims = dims or rt.rt_mlp_dims()
    n_in, n_h, n_out = dims
    stream = torch.cuda.current_stream().cuda_stream
    p = torch.from_numpy(init_params(dims, seed)).cuda()
    off = train_offset(dims)
    n_train = p.numel() - off
    # standardisation from the data (x_mean, x_scale, y_mean, y_scale)
    rt.rt_mlp_colstats(stream, X.data_ptr(), X.shape[0], n_in, p.data_ptr(), p[n_in:].data_ptr(), floor_std)
    rt.rt_mlp_colstats(stream, Y.data_ptr(), Y.shape[0], n_out, p[2 * n_in:].data_ptr(),
                       p[2 * n_in + n_out:].data_ptr(), floor_std)
    g = torch.zeros(n_train, dtype=torch.float32, device="cuda")
    m = torch.zeros_like(g)
    v = torch.zeros_like(g)
    work = torch.empty(rt.rt_mlp_work_floats(n_in, n_h, n_out, batch), dtype=torch.float32, device="cuda")
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    rng = np.random.default_rng(seed)
    n = X.shape[0]
    t = 0
    hist = []
    for ep in range(epochs):
        perm = torch.from_numpy(rng.permutation(n)).cuda()
        Xp, Yp = X[perm].contiguous(), Y[perm].contiguous()
        tot, cnt = 0.0, 0
        for b0 in range(0, n - batch + 1, batch):
            xb, yb = Xp[b0:b0 + batch], Yp[b0:b0 + batch]
            rt.rt_mlp_loss_grad(stream, dims, p.data_ptr(), xb.data_ptr(), yb.data_ptr(), batch, g.data_ptr(),
                                work.data_ptr(), loss.data_ptr())
            t += 1
            rt.rt_mlp_adam(stream, p[off:].data_ptr(), g.data_ptr(), m.data_ptr(), v.data_ptr(), n_train, t, lr)
            tot += float(loss.item())
            cnt += 1
        hist.append(tot / max(1, cnt))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4e}")
    torch.cuda.synchronize()
    return p.cpu().numpy(), hist
