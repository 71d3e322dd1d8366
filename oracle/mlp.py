"""fp64 reference of the schedule-predicting network (test infrastructure only).

The network maps a batch's 32-bin log2 size histogram to one of 12 copy
schedules: 32 -> 64 -> 64 -> 12, ReLU between layers, softmax cross-entropy
on the index of the fastest schedule, Adam updates (Kingma & Ba, ICLR 2015,
Algorithm 1).  Everything is written out from those textbook definitions in
float64 so that a reader can check it by eye; numpy's matmul is the only
library step.

Parameter layout (a flat vector, row-major, shared by name with the GPU
kernels' documented layout): W1[64,32], b1[64], W2[64,64], b2[64],
W3[12,64], b3[12]  -> 7052 values.
"""
import numpy as np

N_IN, N_H, N_OUT = 32, 64, 12
SHAPES = [("W1", (N_H, N_IN)), ("b1", (N_H,)), ("W2", (N_H, N_H)), ("b2", (N_H,)),
          ("W3", (N_OUT, N_H)), ("b3", (N_OUT,))]
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)
assert N_PARAMS == 7052


def unpack(theta: np.ndarray) -> dict:
    out, k = {}, 0
    for name, shape in SHAPES:
        n = int(np.prod(shape))
        out[name] = theta[k:k + n].reshape(shape)
        k += n
    return out


def pack(p: dict) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def features(sizes: np.ndarray) -> np.ndarray:
    """32-bin histogram feature of one batch: bin b counts the requests whose
    size s has floor(log2 s) == b (bins above 31 fold into 31, size 0 into
    bin 0); the feature is log2(1 + count)."""
    counts = np.zeros(N_IN, dtype=np.int64)
    for s in np.asarray(sizes, dtype=np.uint64).tolist():
        b = 0 if s == 0 else min(31, int(s).bit_length() - 1)
        counts[b] += 1
    return np.log2(1.0 + counts.astype(np.float64))


def forward(theta: np.ndarray, x: np.ndarray):
    """Returns logits and the intermediate values the backward pass needs."""
    p = unpack(np.asarray(theta, dtype=np.float64))
    x = np.asarray(x, dtype=np.float64)
    a1 = x @ p["W1"].T + p["b1"]
    h1 = np.maximum(a1, 0.0)
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ p["W3"].T + p["b3"]
    return z, (x, a1, h1, a2, h2)


def softmax(z: np.ndarray) -> np.ndarray:
    m = z.max(axis=1, keepdims=True)
    e = np.exp(z - m)
    return e / e.sum(axis=1, keepdims=True)


def loss(theta: np.ndarray, x: np.ndarray, y: np.ndarray) -> float:
    """Mean softmax cross-entropy: mean_i [ logsumexp(z_i) - z_i[y_i] ]."""
    z, _ = forward(theta, x)
    m = z.max(axis=1)
    lse = m + np.log(np.exp(z - m[:, None]).sum(axis=1))
    return float(np.mean(lse - z[np.arange(len(y)), y]))


def grad(theta: np.ndarray, x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """Gradient of ``loss`` by the chain rule, layer by layer."""
    z, (x, a1, h1, a2, h2) = forward(theta, x)
    p = unpack(np.asarray(theta, dtype=np.float64))
    B = x.shape[0]
    dz = softmax(z)
    dz[np.arange(B), y] -= 1.0
    dz /= B
    g = {}
    g["W3"] = dz.T @ h2
    g["b3"] = dz.sum(axis=0)
    dh2 = dz @ p["W3"]
    da2 = dh2 * (a2 > 0)
    g["W2"] = da2.T @ h1
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ p["W2"]
    da1 = dh1 * (a1 > 0)
    g["W1"] = da1.T @ x
    g["b1"] = da1.sum(axis=0)
    return pack(g)


class Adam:
    """Adam with bias correction; state m, v start at zero, step t from 1."""

    def __init__(self, n: int, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
        self.m = np.zeros(n)
        self.v = np.zeros(n)
        self.t = 0
        self.lr, self.b1, self.b2, self.eps = lr, beta1, beta2, eps

    def step(self, theta: np.ndarray, g: np.ndarray) -> np.ndarray:
        self.t += 1
        self.m = self.b1 * self.m + (1.0 - self.b1) * g
        self.v = self.b2 * self.v + (1.0 - self.b2) * g * g
        mhat = self.m / (1.0 - self.b1 ** self.t)
        vhat = self.v / (1.0 - self.b2 ** self.t)
        return theta - self.lr * mhat / (np.sqrt(vhat) + self.eps)


def predict(theta: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Class with the largest logit; ties go to the lowest index."""
    z, _ = forward(theta, np.atleast_2d(x))
    return np.argmax(z, axis=1)
