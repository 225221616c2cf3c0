"""3-D convolutional network of the learned PCG initial guess -- oracle.

Test infrastructure only (see the package docstring).

Four 3x3x3 convolutions with zero padding 1 on a lattice of shape
(nz, ny, nx) (x fastest, the node numbering of the Kuhn mesh), channels
3 -> 16 -> 16 -> 16 -> 1, ReLU after the first three. Written directly from
the definition of a cross-correlation:

    z[c_out, v] = b[c_out] + sum_{tap, c_in} w[c_out, c_in, tap] x[c_in, v + tap]

with x taken as 0 outside the lattice; taps run over (dz, dy, dx) in
{-1, 0, 1}^3 with dx fastest. Forward, loss (mean squared error) and the
gradients with respect to the inputs, weights and biases, all in FP64.
"""
import numpy as np

TAPS = [(dz, dy, dx) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
CHANNELS = (3, 16, 16, 16, 1)


def shift(x, dz, dy, dx):
    """y[..., z, y, x] = x[..., z + dz, y + dy, x + dx], zero outside."""
    out = np.zeros_like(x)
    nz, ny, nx = x.shape[-3:]

    def sl(d, n):
        return (slice(max(-d, 0), n - max(d, 0)), slice(max(d, 0), n - max(-d, 0)))

    (oz, iz), (oy, iy), (ox, ix) = sl(dz, nz), sl(dy, ny), sl(dx, nx)
    out[..., oz, oy, ox] = x[..., iz, iy, ix]
    return out


def conv(x, w, b):
    """x [C_in, nz, ny, nx], w [C_out, C_in, 27], b [C_out] -> [C_out, nz, ny, nx]."""
    z = np.zeros((w.shape[0],) + x.shape[1:])
    for t, (dz, dy, dx) in enumerate(TAPS):
        xs = shift(x, dz, dy, dx)
        z += np.einsum("oi,i...->o...", w[:, :, t], xs)
    return z + b[:, None, None, None]


def conv_grad(x, w, dz_out):
    """Gradients of sum(dz_out * conv(x, w, b)) w.r.t. x, w and b."""
    dx = np.zeros_like(x)
    dw = np.zeros_like(w)
    for t, (dz, dy, dxx) in enumerate(TAPS):
        xs = shift(x, dz, dy, dxx)
        dw[:, :, t] = dz_out.reshape(dz_out.shape[0], -1) @ xs.reshape(xs.shape[0], -1).T
        # x[v + tap] feeds z[v]: its gradient is dz_out shifted back
        dx += shift(np.einsum("oi,o...->i...", w[:, :, t], dz_out), -dz, -dy, -dxx)
    db = dz_out.sum(axis=(1, 2, 3))
    return dx, dw, db


def init_params(rng):
    """He-style initial weights, zero biases."""
    params = []
    for cin, cout in zip(CHANNELS[:-1], CHANNELS[1:]):
        w = rng.standard_normal((cout, cin, 27)) * np.sqrt(2.0 / (27 * cin))
        params.append([w, np.zeros(cout)])
    return params


def forward(params, x):
    """Returns the output [nz, ny, nx] and the list of layer inputs."""
    acts = [x]
    h = x
    for i, (w, b) in enumerate(params):
        z = conv(h, w, b)
        h = np.maximum(z, 0.0) if i < len(params) - 1 else z
        acts.append(h)
    return h[0], acts


def loss_and_grads(params, x, target):
    """L = mean((y - target)^2) and dL/d(params) by backpropagation."""
    y, acts = forward(params, x)
    V = y.size
    L = np.mean((y - target) ** 2)
    g = (2.0 / V) * (y - target)[None]
    grads = [None] * len(params)
    for i in range(len(params) - 1, -1, -1):
        w, b = params[i]
        dx, dw, db = conv_grad(acts[i], w, g)
        grads[i] = [dw, db]
        if i > 0:
            g = dx * (acts[i] > 0)          # ReLU of the previous layer
    return L, grads
