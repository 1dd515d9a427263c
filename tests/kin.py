"""Small kinematic helpers for the oracle pins (boosts and rotations)."""
import numpy as np


def boost(p, beta):
    """Boost four-vectors p[..., 4] by velocity beta[3] (beta < 1)."""
    beta = np.asarray(beta, dtype=np.float64)
    b2 = beta @ beta
    gamma = 1.0 / np.sqrt(1.0 - b2)
    bp = p[..., 1:] @ beta
    out = np.empty_like(p)
    out[..., 0] = gamma * (p[..., 0] + bp)
    coef = (gamma - 1.0) * bp / b2 + gamma * p[..., 0]
    out[..., 1:] = p[..., 1:] + coef[..., None] * beta
    return out


def rotation(axis, angle):
    axis = np.asarray(axis, dtype=np.float64)
    axis = axis / np.linalg.norm(axis)
    k = np.array([[0, -axis[2], axis[1]], [axis[2], 0, -axis[0]], [-axis[1], axis[0], 0]])
    return np.eye(3) + np.sin(angle) * k + (1 - np.cos(angle)) * (k @ k)


def rotate(p, r):
    out = p.copy()
    out[..., 1:] = p[..., 1:] @ r.T
    return out


def boost_from_rest(p_rest, q):
    """Take p_rest given in the rest frame of q to the frame where q is given."""
    out = np.empty(np.broadcast_shapes(p_rest.shape, q.shape))
    for i in range(q.shape[0]):
        beta = q[i, 1:] / q[i, 0]
        out[i] = boost(p_rest[i], beta) if beta @ beta > 0 else p_rest[i]
    return out


def mdot(a, b):
    return a[..., 0] * b[..., 0] - np.sum(a[..., 1:] * b[..., 1:], axis=-1)
