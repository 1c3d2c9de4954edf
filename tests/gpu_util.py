"""Helpers for the GPU tests: device transfer and the oracle reference of
each phase on the same seeded inputs."""
import numpy as np

from oracle import moduli as md
from oracle import scheme


def cuda_ok():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def host(t):
    return t.detach().cpu().numpy()


def oracle_shifts(A, B, moduli, mode):
    """(s, t) as the library reports them: the oracle's shifts, with the
    non-finite marker on rows/columns holding a NaN or an infinity."""
    s, t, finA, finB, _ = scheme._shifts(A, B, moduli, mode)
    s = np.where(finA, s, -(2 ** 31))
    t = np.where(finB, t, -(2 ** 31))
    return s.astype(np.int64), t.astype(np.int64)


def plane_offsets(rows: int, k_pad: int) -> np.ndarray:
    """Byte offset of every entry (row, h) of a residue plane in the
    library's GEMM block order (layout documented in include/ozemu.h)."""
    r = np.arange(rows, dtype=np.int64)[:, None]
    h = np.arange(k_pad, dtype=np.int64)[None, :]
    rr = r % 256
    return (((r // 256) * (k_pad // 64) + h // 64) * 16384 + rr * 64
            + ((((h % 64) // 16) ^ ((rr // 4) % 4)) * 16) + h % 16)


def to_blocked(P: np.ndarray) -> np.ndarray:
    """[N, rows, k_pad] row-major planes -> the same bytes in block order."""
    N, R, K = P.shape
    off = plane_offsets(R, K).ravel()
    out = np.empty((N, R * K), dtype=P.dtype)
    for l in range(N):
        out[l, off] = P[l].ravel()
    return out.reshape(N, R, K)


def from_blocked(Q: np.ndarray) -> np.ndarray:
    """Inverse of to_blocked."""
    N, R, K = Q.shape
    off = plane_offsets(R, K)
    return np.stack([Q[l].ravel()[off] for l in range(N)])


def oracle_planes(A, B, moduli, mode, pads):
    """Zero-padded int8 residue planes [N, m_pad, k_pad], [N, n_pad, k_pad]."""
    mp, np_, kp = pads
    s, t, finA, finB, _ = scheme._shifts(A, B, moduli, mode)
    Af, Bf, _, _ = scheme._finite_parts(A, B)
    Ai = scheme.truncate(Af, s, 1)
    Bi = scheme.truncate(Bf, t, 0)
    m, k = A.shape
    n = B.shape[1]
    PA = np.zeros((len(moduli), mp, kp), dtype=np.int8)
    PB = np.zeros((len(moduli), np_, kp), dtype=np.int8)
    for l, mm in enumerate(moduli):
        PA[l, :m, :k] = scheme.balanced_residues(Ai, int(mm))
        PB[l, :n, :k] = scheme.balanced_residues(Bi, int(mm)).T
    return PA, PB


def default_moduli(n):
    return md.best_coprime_set(n, 256)
