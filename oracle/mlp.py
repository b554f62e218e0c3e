"""Plain FP64 reference of the kappa-coefficient surrogate network.

TEST INFRASTRUCTURE ONLY (part of the CPU oracle): used by the tests to check
the GPU forward pass, the GPU backward pass and the GPU training kernels.

The network, as the library defines it (restated here from that definition,
not shared with it):
    features x = ((kappa - 5.5)/2.5, (log10 w - 0.75)/1.25, (log10 X - 2.5)/4.5, cos theta)
    h1 = silu(W1 x + b1), h2 = silu(W2 h1 + b2), h3 = silu(W3 h2 + b3)
    z = W4 h3 + b4,  log10 I_k = sum_j c_kj m_j(x) + mu_k + sd_k z_k,  silu(t) = t / (1 + e^-t)
with m_j the 20 monomials of degree <= 3 in (x0, x1, x2) (order: 1, x0, x1,
x2, then the degree-2 and degree-3 products with non-decreasing indices)
with the weight matrices rounded to bfloat16 (round to nearest, ties to
even) and the biases used as they are.  Parameter vector (9160 floats):
W1[64][4], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[8][64], b4[8].
Normalisation vector (176): mu[8], sd[8], c[8][20].
Loss over n samples: L = sum (z - t)^2 / (8 n), t = (log10 I - baseline - mu) / sd.
The backward pass below is the chain rule written out by hand; the tests
check it against finite differences of the forward pass.
"""
import numpy as np

H = 64
SHAPES = [("W1", (H, 4)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
          ("W4", (8, H)), ("b4", (8,))]
NPARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def bf16_round(a):
    """Round float32 values to bfloat16 (nearest, ties to even); float64 out."""
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    return u.view(np.float32).astype(np.float64)


def unpack(params, rounded=True):
    """Parameter vector -> dict of FP64 arrays (weights bf16-rounded when asked)."""
    p = np.asarray(params)
    out, off = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        v = p[off:off + n]
        if name.startswith("W") and rounded:
            v = bf16_round(v.astype(np.float32))
        out[name] = np.asarray(v, dtype=np.float64).reshape(shape)
        off += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def features(inp):
    """Feature rows, rounded to FP32 as the library forms them."""
    inp = np.asarray(inp, dtype=np.float64)
    f = np.stack([(inp[:, 0] - 5.5) / 2.5, (np.log10(inp[:, 1]) - 0.75) / 1.25, (np.log10(inp[:, 2]) - 2.5) / 4.5,
                  inp[:, 3]], axis=1)
    return f.astype(np.float32).astype(np.float64)


def monomials(f):
    """The 20 monomials of degree <= 3 in the first three features."""
    import itertools
    cols = [np.ones(f.shape[0])]
    for deg in (1, 2, 3):
        for c in itertools.combinations_with_replacement(range(3), deg):
            cols.append(np.prod(f[:, list(c)], axis=1))
    return np.stack(cols, axis=1)


def _sig(z):
    return 1.0 / (1.0 + np.exp(-z))


def forward_z(W, x):
    """Standardised outputs z [n, 8] and the pre-activations of the hidden layers."""
    z1 = x @ W["W1"].T + W["b1"]
    h1 = z1 * _sig(z1)
    z2 = h1 @ W["W2"].T + W["b2"]
    h2 = z2 * _sig(z2)
    z3 = h2 @ W["W3"].T + W["b3"]
    h3 = z3 * _sig(z3)
    z = h3 @ W["W4"].T + W["b4"]
    return z, (x, z1, h1, z2, h2, z3, h3)


def predict_log10(params, norm, inp):
    """log10 of the eight integrals predicted for inputs [n, 4]."""
    W = unpack(params)
    f = features(inp)
    z, _ = forward_z(W, f)
    norm = np.asarray(norm, dtype=np.float64)
    base = monomials(f) @ norm[16:].reshape(8, 20).T
    return base + norm[:8] + norm[8:16] * z


def loss_and_grad(params, norm, inp, integ, rounded=True):
    """Loss and its gradient with respect to the parameter vector (weights
    enter rounded; the gradient passes straight through the rounding)."""
    W = unpack(params, rounded=rounded)
    norm = np.asarray(norm, dtype=np.float64)
    f = features(inp)
    base = monomials(f) @ norm[16:].reshape(8, 20).T
    t = (np.log10(np.asarray(integ, dtype=np.float64)) - base - norm[:8]) / norm[8:16]
    z, (x, z1, h1, z2, h2, z3, h3) = forward_z(W, f)
    n = x.shape[0]
    d = z - t
    loss = float(np.sum(d * d) / (8.0 * n))
    dz = 2.0 * d / (8.0 * n)

    def dsilu(a):
        s = _sig(a)
        return s * (1.0 + a * (1.0 - s))

    g = {"W4": dz.T @ h3, "b4": dz.sum(0)}
    d3 = (dz @ W["W4"]) * dsilu(z3)
    g["W3"] = d3.T @ h2
    g["b3"] = d3.sum(0)
    d2 = (d3 @ W["W3"]) * dsilu(z2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ W["W2"]) * dsilu(z1)
    g["W1"] = d1.T @ x
    g["b1"] = d1.sum(0)
    return loss, pack(g)
