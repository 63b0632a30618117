"""FP64 CPU oracle of the surrogate network -- TEST INFRASTRUCTURE.

Only the tests, smoke() and bench.py's cpu_baseline may use this module.

The network maps features x (53 values: 24 momentum components divided by
sqrt(s)/2, (kappa-1)/0.2, and for 14 particle pairs 2 p_i.p_j/s and its
logarithm) through four hidden layers a_l = SiLU(W_l a_{l-1}
+ b_l) of width 256 to h = w5 . a_4 + b5, and predicts
yhat = (kappa - 1) h for y = log(|M_kappa|^2 / |M_base|^2).  The loss is the
mean squared error.  Gradients are written out by the chain rule.

With bf16=True the forward and backward passes round to bfloat16 (nearest
even) at the points where the GPU kernels store bfloat16 values: the
features, the hidden-layer weights W1..W4, every post-activation a_l, and every
back-propagated dz_l; everything else stays in float64.  This lets the GPU
gradients be compared at float32-accumulation accuracy.

Flat parameter layout (float32 on the device): W1[256][64] (input columns
53..63 unused), b1, W2[256][256], b2, W3, b3, W4, b4, w5[256], b5.
"""
import numpy as np

H = 256
K0 = 64
NFEAT = 53
SIZES = [("W1", (H, K0)), ("b1", (H,)), ("W2", (H, H)), ("b2", (H,)), ("W3", (H, H)), ("b3", (H,)),
         ("W4", (H, H)), ("b4", (H,)), ("w5", (H,)), ("b5", (1,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SIZES)


def unpack(flat):
    flat = np.asarray(flat, dtype=np.float64)
    assert flat.size == N_PARAMS
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = flat[o:o + n].reshape(shape)
        o += n
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).reshape(-1) for name, _ in SIZES])


def bf16(a):
    """Round to bfloat16 (nearest even) through float32, returned as float64."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def sigmoid(z):
    return 1.0 / (1.0 + np.exp(-z))


def silu(z):
    return z * sigmoid(z)


def dsilu(z):
    s = sigmoid(z)
    return s * (1.0 + z * (1.0 - s))


def forward(params, x, kd, emulate_bf16=False):
    """x [m, 25], kd [m]; returns (yhat, cache)."""
    p = unpack(params)
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a = np.zeros((x.shape[0], K0))
    a[:, :NFEAT] = x
    a = r(a)
    acts, zs = [a], []
    for l in range(1, 5):
        W = r(p[f"W{l}"])
        z = a @ W.T + p[f"b{l}"]
        a = r(silu(z))
        zs.append(z)
        acts.append(a)
    h = a @ p["w5"] + p["b5"][0]
    yhat = kd * h
    return yhat, dict(acts=acts, zs=zs, p=p, kd=kd)


def loss_and_grad(params, x, kd, y, emulate_bf16=False):
    """Mean squared error and its gradient (flat, same layout as params)."""
    r = bf16 if emulate_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    yhat, c = forward(params, x, kd, emulate_bf16)
    m = x.shape[0]
    diff = yhat - y
    loss = np.mean(diff ** 2)
    p, acts, zs = c["p"], c["acts"], c["zs"]
    g = {}
    dh = 2.0 * diff / m * kd                       # d loss / d h
    g["w5"] = acts[4].T @ dh
    g["b5"] = np.array([dh.sum()])
    dz = r(np.outer(dh, p["w5"]) * dsilu(zs[3]))   # layer 4
    for l in range(4, 0, -1):
        g[f"W{l}"] = dz.T @ acts[l - 1]
        g[f"b{l}"] = dz.sum(axis=0)
        if l > 1:
            da = dz @ r(p[f"W{l}"])
            dz = r(da * dsilu(zs[l - 2]))
    return loss, yhat, pack(g)


def features(mom, kappa):
    """Feature rows (event-major, point-minor) of SoA momenta mom [n_ext, 4, n]."""
    n_ext, _, n = mom.shape
    rs = mom[0, 0] + mom[1, 0]
    P = len(kappa)
    x = np.zeros((n, P, NFEAT))
    comps = (mom.reshape(n_ext * 4, n) * (2.0 / rs)).T
    x[:, :, :min(24, n_ext * 4)] = comps[:, None, :24]
    x[:, :, 24] = ((np.asarray(kappa) - 1.0) / 0.2)[None, :]
    c = 25
    for i in range(6):
        for j in range(i + 1, 6):
            if (i, j) == (0, 1):
                continue
            if j < n_ext:
                pi, pj = mom[i], mom[j]
                u = 2.0 * (pi[0] * pj[0] - pi[1] * pj[1] - pi[2] * pj[2] - pi[3] * pj[3]) / rs ** 2
                x[:, :, c] = u[:, None]
                x[:, :, c + 14] = np.log(np.maximum(u, 1e-12))[:, None]
            c += 1
    kd = np.broadcast_to(np.asarray(kappa) - 1.0, (n, P))
    return x.reshape(n * P, NFEAT), kd.reshape(n * P).copy()


def init_params(seed=1, scale=1.0):
    """Random parameters with the same shapes as the device network (for tests)."""
    rng = np.random.default_rng(seed)
    d = {}
    d["W1"] = np.zeros((H, K0))
    d["W1"][:, :NFEAT] = rng.uniform(-1, 1, (H, NFEAT)) * np.sqrt(6 / NFEAT) * scale
    for l in (2, 3, 4):
        d[f"W{l}"] = rng.uniform(-1, 1, (H, H)) * np.sqrt(6 / H) * scale
    for l in (1, 2, 3, 4):
        d[f"b{l}"] = rng.uniform(-0.1, 0.1, H)
    d["w5"] = rng.uniform(-1, 1, H) / np.sqrt(H)
    d["b5"] = np.array([0.05])
    return pack(d)
