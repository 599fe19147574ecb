"""TEST INFRASTRUCTURE ONLY -- plain reference of the learned proposal.

A RealNVP-style flow of affine coupling layers on the 11 standardized
parameters, the negative log-likelihood it is trained on, its gradient by
plain back-propagation, and the Adam update (Kingma & Ba 2015).  FP64 numpy,
one sample at a time conceptually (written with batch arrays for speed, no
fusion).  The GPU library computes in BF16/FP32; this reference takes the
same BF16-rounded weights and, with ``rnd=True``, rounds the three
matrix-product inputs of every conditioner network to BF16 at the same
points, so both sides evaluate the same function up to FP32 accumulation.
Shares no code with the GPU library.

Conventions (the paper gives none; these are the proposal's definition):
  u = float32(L^-1 (theta - mu)) with L lower triangular (a whitening map:
  L L^T is a covariance; a vector sigma stands for L = diag(sigma)), the
  triangular solve by forward substitution in FP64; base density N(0, I_11).
  8 layers.  Layer 2p conditions on C_p = {i : (i + 3p) mod 11 < 6} (6
  entries) and transforms the other 5; layer 2p + 1 conditions on those 5
  and transforms C_p.  Conditioner: x_C -> 256 (ReLU) -> 256 (ReLU) -> 2 n_T
  (linear), first n_T outputs s_hat, last n_T outputs t;
  s = 3 tanh(s_hat / 3).
  Normalizing direction (u -> z), layers 0..7: y_T = x_T exp(s) + t,
  y_C = x_C, log det += sum s.
  log q_u(u) = -|z|^2 / 2 - (11/2) log(2 pi) + log det;
  log q(theta) = log q_u(u) - sum log L_ii.
  A temperature tau widens the base density to N(0, tau^2 I): draws use
  z = tau * (standard normal), rounded to FP32 after the product, and
  log q_u(u) = -|z|^2 / (2 tau^2) - 11 log tau - (11/2) log(2 pi) + log det.
  Parameters per layer, y = x W + b: W1 [n_C, 256], b1 [256], W2 [256, 256],
  b2 [256], W3 [256, 2 n_T], b3 [2 n_T]; stored flat in that order, layer
  after layer (562264 numbers).
"""
import math

import numpy as np

D = 11
HID = 256
N_LAYERS = 8
S_MAX = 3.0


def cond_set(layer):
    """Indices the layer conditions on (sorted)."""
    p = layer // 2
    c = [i for i in range(D) if (i + 3 * p) % D < 6]
    if layer % 2:
        c = [i for i in range(D) if i not in c]
    return c


def trans_set(layer):
    c = cond_set(layer)
    return [i for i in range(D) if i not in c]


def shapes(layer):
    nc, nt = len(cond_set(layer)), len(trans_set(layer))
    return [("W1", (nc, HID)), ("b1", (HID,)), ("W2", (HID, HID)), ("b2", (HID,)),
            ("W3", (HID, 2 * nt)), ("b3", (2 * nt,))]


def n_params():
    return sum(int(np.prod(s)) for l in range(N_LAYERS) for _, s in shapes(l))


def unflatten(flat):
    """Flat parameter vector -> list of per-layer dicts (views)."""
    out, o = [], 0
    for l in range(N_LAYERS):
        d = {}
        for name, s in shapes(l):
            n = int(np.prod(s))
            d[name] = flat[o:o + n].reshape(s)
            o += n
        out.append(d)
    assert o == flat.size
    return out


def bf16(x):
    """Round to the nearest BF16 value (ties to even), returned as float64.
    Works on the float32 bit pattern: keep the top 16 bits after adding
    0x7FFF plus the lowest kept bit."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> 16) & 1
    r = ((b + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).astype(np.float64)
    nan = np.isnan(f)
    if np.any(nan):
        out = np.where(nan, np.nan, out)
    return out


def init_params(seed, scale_out=0.0):
    """Float32 parameters: Kaiming-uniform hidden layers, output layer scaled
    by scale_out (0 gives the identity map)."""
    rng = np.random.default_rng(seed)
    flat = np.zeros(n_params(), dtype=np.float32)
    for d, l in zip(unflatten(flat), range(N_LAYERS)):
        for name in ("W1", "W2"):
            fan_in = d[name].shape[0]
            bound = math.sqrt(6.0 / fan_in)
            d[name][...] = rng.uniform(-bound, bound, size=d[name].shape)
        d["W3"][...] = scale_out * rng.uniform(-1, 1, size=d["W3"].shape) / math.sqrt(HID)
    return flat


def _weights(p, k, rnd):
    """W_k (BF16-rounded with rnd) and b_k of a layer's parameter dict, FP64."""
    W = p["W%d" % k]
    W = bf16(W) if rnd else np.asarray(W, dtype=np.float64)
    return W, np.asarray(p["b%d" % k], dtype=np.float64)


def _dense(p, k, a, rnd):
    """a W_k + b_k and |a| |W_k| + |b_k| (the scale of the sum's rounding error
    in any accumulation order)."""
    W, b = _weights(p, k, rnd)
    a = np.asarray(a, dtype=np.float64)
    return a @ W + b, np.abs(a) @ np.abs(W) + np.abs(b)


def dense(flat, l, k, a, rnd=True):
    """Product k (1, 2 or 3) of layer l's conditioner on its input rows a."""
    return _dense(unflatten(np.asarray(flat))[l], k, a, rnd)


def _net(p, xc, rnd):
    """Conditioner forward; returns (s, t, cache)."""
    r = bf16 if rnd else (lambda a: np.asarray(a, dtype=np.float64))
    a0 = r(xc)
    a1 = r(np.maximum(_dense(p, 1, a0, rnd)[0], 0.0))
    a2 = r(np.maximum(_dense(p, 2, a1, rnd)[0], 0.0))
    o = _dense(p, 3, a2, rnd)[0]
    nt = o.shape[1] // 2
    th = np.tanh(o[:, :nt] / S_MAX)
    s = S_MAX * th
    t = o[:, nt:]
    W1, W2, W3 = (_weights(p, k, rnd)[0] for k in (1, 2, 3))
    return s, t, (a0, a1, a2, W1, W2, W3, th, o)


def coupling(l, x, o, inverse=False):
    """Affine update of layer l on the rows x given its conditioner output o
    [n, 2 n_T] = (s_hat, t): s = 3 tanh(s_hat / 3); normalizing y_T = x_T e^s + t,
    inverse x_T = (y_T - t) e^-s.  Returns (new rows, sum of s per row)."""
    T = trans_set(l)
    nt = len(T)
    s = S_MAX * np.tanh(np.asarray(o[:, :nt], dtype=np.float64) / S_MAX)
    t = np.asarray(o[:, nt:2 * nt], dtype=np.float64)
    y = np.array(x, dtype=np.float64)
    y[:, T] = (y[:, T] - t) * np.exp(-s) if inverse else y[:, T] * np.exp(s) + t
    return y, s.sum(axis=1)


def layer(flat, l, x, inverse=False, rnd=True):
    """One coupling layer l on the rows x [n, 11]; returns (new rows, sum of s
    per row)."""
    p = unflatten(np.asarray(flat))[l]
    x = np.asarray(x, dtype=np.float64)
    *_, cache = _net(p, x[:, cond_set(l)], rnd)
    return coupling(l, x, cache[-1], inverse)


def layer_order(inverse=False):
    """Layers in the order a pass applies them."""
    return list(reversed(range(N_LAYERS))) if inverse else list(range(N_LAYERS))


def trace(flat, x0, inverse=False, rnd=True):
    """A pass with its intermediates: the rows before the first layer and after
    each layer in the order applied (states [9, n, 11]), the running sum of s at
    the same points ([9, n]), and for each layer l (by index) its conditioner
    stages a0, a1, a2 (network input and the two hidden layers, BF16-rounded
    with rnd) and o (output)."""
    layers = unflatten(np.asarray(flat))
    x = np.array(x0, dtype=np.float64)
    st, ld = [x.copy()], [np.zeros(x.shape[0])]
    acts = [None] * N_LAYERS
    for l in layer_order(inverse):
        *_, cache = _net(layers[l], x[:, cond_set(l)], rnd)
        acts[l] = dict(a0=cache[0], a1=cache[1], a2=cache[2], o=cache[-1])
        x, s = coupling(l, x, cache[-1], inverse)
        st.append(x.copy())
        ld.append(ld[-1] + s)
    return np.stack(st), np.stack(ld), acts


def states(flat, x0, inverse=False, rnd=True):
    """(states [9, n, 11], running sum of s [9, n]) of a pass (see trace)."""
    st, ld, _ = trace(flat, x0, inverse, rnd)
    return st, ld


def forward(flat, u, rnd=True):
    """Normalizing direction: u [n, 11] -> (z [n, 11], log det [n])."""
    st, ld = states(flat, u, False, rnd)
    return st[-1], ld[-1]


def inverse(flat, z, rnd=True):
    """Generative direction: z -> (u, log det of the normalizing map at u)."""
    st, ld = states(flat, z, True, rnd)
    return st[-1], ld[-1]


def log_base(z, logdet, tau=1.0):
    """log q_u from the latent rows z and the normalizing map's log det:
    log N(z; 0, tau^2 I) + log det."""
    z = np.asarray(z, dtype=np.float64)
    return (-0.5 * (z * z).sum(axis=1) / (tau * tau) - D * math.log(tau)
            - 0.5 * D * math.log(2.0 * math.pi) + np.asarray(logdet, dtype=np.float64))


def log_prob_u(flat, u, rnd=True, tau=1.0):
    z, ld = forward(flat, u, rnd)
    return log_base(z, ld, tau)


def whitening(sigma):
    """L from a vector of scales (diagonal) or a lower-triangular matrix."""
    s = np.asarray(sigma, dtype=np.float64)
    return np.diag(s) if s.ndim == 1 else np.tril(s)


def standardize(theta, mu, sigma):
    """u = float32(L^-1 (theta - mu)), forward substitution row by row."""
    L = whitening(sigma)
    r = np.atleast_2d(np.asarray(theta, dtype=np.float64)) - mu
    u = np.zeros_like(r)
    for k in range(D):
        acc = r[:, k].copy()
        for j in range(k):
            acc -= L[k, j] * u[:, j]
        u[:, k] = acc / L[k, k]
    return u.astype(np.float32).astype(np.float64)


def unstandardize(u, mu, sigma):
    return mu + np.asarray(u, dtype=np.float64) @ whitening(sigma).T


def log_prob(flat, theta, mu, sigma, rnd=True, tau=1.0):
    """log q(theta) of the proposal."""
    return (log_prob_u(flat, standardize(theta, mu, sigma), rnd, tau)
            - np.log(np.diag(whitening(sigma))).sum())


def nll_and_grad(flat, u, weight=None, rnd=True):
    """NLL = sum_i w_i (|z_i|^2/2 + 11/2 log 2 pi - log det_i), w_i = 1/n by
    default, and its gradient with respect to the flat parameters (the
    BF16 roundings pass gradients unchanged)."""
    layers = unflatten(np.asarray(flat))
    n = u.shape[0]
    w = np.full(n, 1.0 / n) if weight is None else np.asarray(weight, dtype=np.float64)
    x = np.array(u, dtype=np.float64)
    logdet = np.zeros(n)
    tape = []
    for l, p in enumerate(layers):
        C, T = cond_set(l), trans_set(l)
        xin = x.copy()
        s, t, cache = _net(p, x[:, C], rnd)
        x[:, T] = x[:, T] * np.exp(s) + t
        logdet += s.sum(axis=1)
        tape.append((xin, s, cache))
    nll = float(np.sum(w * (0.5 * (x * x).sum(axis=1) + 0.5 * D * math.log(2.0 * math.pi) - logdet)))
    grads = [dict() for _ in range(N_LAYERS)]
    gy = w[:, None] * x                      # d NLL / d z
    gld = -w                                 # d NLL / d log det
    for l in reversed(range(N_LAYERS)):
        C, T = cond_set(l), trans_set(l)
        xin, s, (a0, a1, a2, W1, W2, W3, th, _) = tape[l]
        es = np.exp(s)
        gyT = gy[:, T]
        gx = gy.copy()
        gx[:, T] = gyT * es
        gs = gyT * xin[:, T] * es + gld[:, None]
        gt = gyT
        gshat = gs * (1.0 - th * th)
        go = np.concatenate([gshat, gt], axis=1)
        g = grads[l]
        g["W3"] = a2.T @ go
        g["b3"] = go.sum(axis=0)
        ga2 = (go @ W3.T) * (a2 > 0)
        g["W2"] = a1.T @ ga2
        g["b2"] = ga2.sum(axis=0)
        ga1 = (ga2 @ W2.T) * (a1 > 0)
        g["W1"] = a0.T @ ga1
        g["b1"] = ga1.sum(axis=0)
        gx[:, C] += ga1 @ W1.T
        gy = gx
    out = np.zeros(flat.size)
    o = 0
    for l in range(N_LAYERS):
        for name, sh in shapes(l):
            k = int(np.prod(sh))
            out[o:o + k] = grads[l][name].ravel()
            o += k
    return nll, out


def adam_step(p, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (step number t >= 1) of p in place; returns (p, m, v)."""
    m[...] = beta1 * m + (1.0 - beta1) * g
    v[...] = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    p[...] = p - lr * mh / (np.sqrt(vh) + eps)
    return p, m, v
