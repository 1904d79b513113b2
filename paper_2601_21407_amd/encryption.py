"""HH encryption (Results, accessible exploration of biological neuron
models; Methods, HH encryption): a filter bank of HH neurons that differ
in their time constant tau maps a sinusoidal input (f, A) to an n-bit code
(bit k: the neuron with taus[k] fires within the response window), and a
key of 2^n (f, A) pairs, one per code, defines the substitution tables:
B[k] = code of key[k] (the bank's response, evaluated by simulation) and
A = B^-1.  Plaintext is cut into n-bit segments and chained (CBC):
c_i = A[p_i xor c_{i-1}]; decryption simulates the bank on key[c_i] and
takes p_i = B[c_i] xor c_{i-1}.

Every neuron of the bank runs in libhh's step kernel (sinusoidal input
mode); this module builds the populations and does the byte logic.
"""
from __future__ import annotations

import numpy as np
import torch

from . import hh
from . import workloads as W


def bank_levels(model: dict, taus, freqs, amps, T: int, window: int, dev: str = "cuda",
                timing: dict | None = None):
    """Steps at or above threshold within the last `window` of T steps, for
    every (input, bank neuron): [P][n_taus].  Neuron p * n_taus + k gets
    input (freqs[p], amps[p]) and time constant taus[k]: the bank is the
    model's per-neuron dimension (N = n_taus) and the inputs its batch
    (B = P), so the time constants' coefficients are stored once.  timing:
    filled with the simulation's kernel time in ms."""
    nb = len(taus)
    P = len(freqs)
    coef = W.timescale_coef(model, taus)
    M = hh.Model(model, nb, P, coef=torch.tensor(coef, device=dev))
    amp = torch.tensor(np.repeat(np.asarray(amps, np.float32), nb), device=dev)
    fr = torch.tensor(np.repeat(np.asarray(freqs, np.float32), nb), device=dev)
    st = M.new_state()
    M.init_state(st, v0_scalar=-65.0)
    lvl = torch.zeros(P * nb, device=dev)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    if T > window:
        M.step_n(st, T - window, 0, sine=(amp, fr))
    M.step_n(st, window, T - window, sine=(amp, fr), level=lvl)
    e1.record()
    status, bad = M.check()
    if status != 0:
        raise RuntimeError("filter bank simulation failed (%d at %d)" % (status, bad))
    if timing is not None:
        timing["ms"] = e0.elapsed_time(e1)
    return lvl.cpu().numpy().reshape(P, nb)


def codes_from_levels(levels: np.ndarray) -> np.ndarray:
    """The bank's n-bit code: bit k set when neuron k reached threshold."""
    bits = (np.asarray(levels) > 0).astype(np.int64)
    return (bits << np.arange(bits.shape[1])).sum(axis=1)


def make_key(model: dict, taus, freqs, amps, rng, T: int, window: int):
    """Evaluate the bank on the (freqs x amps) grid and draw the key: for a
    random order of the 2^n codes, one grid point per code among those whose
    four grid neighbours give the same code (away from the region borders).
    Returns (key_f, key_A, B) with B[k] the code of key[k]."""
    nb = len(taus)
    F, A = np.meshgrid(np.asarray(freqs, np.float64), np.asarray(amps, np.float64))
    codes = codes_from_levels(bank_levels(model, taus, F.ravel(), A.ravel(), T, window))
    C = codes.reshape(F.shape)
    inner = np.zeros_like(C, dtype=bool)
    inner[1:-1, 1:-1] = ((C[1:-1, 1:-1] == C[:-2, 1:-1]) & (C[1:-1, 1:-1] == C[2:, 1:-1]) &
                         (C[1:-1, 1:-1] == C[1:-1, :-2]) & (C[1:-1, 1:-1] == C[1:-1, 2:]))
    B = rng.permutation(1 << nb)
    key_f, key_A = np.zeros(1 << nb), np.zeros(1 << nb)
    for k, code in enumerate(B):
        cand = np.argwhere(inner & (C == code))
        if len(cand) == 0:
            raise ValueError("code %d is not reachable on this grid with taus %s" % (code, list(taus)))
        i, j = cand[rng.integers(len(cand))]
        key_f[k], key_A[k] = F[i, j], A[i, j]
    return key_f, key_A, B


def to_segments(data: bytes, nb: int) -> np.ndarray:
    """Bytes to n-bit segments, low bits first (nb divides 8)."""
    if 8 % nb:
        raise ValueError("segment width must divide 8")
    b = np.frombuffer(bytes(data), dtype=np.uint8).astype(np.int64)
    sh = np.arange(0, 8, nb)
    return ((b[:, None] >> sh[None, :]) & ((1 << nb) - 1)).ravel()


def from_segments(seg: np.ndarray, nb: int) -> bytes:
    s = np.asarray(seg, np.int64).reshape(-1, 8 // nb)
    sh = np.arange(0, 8, nb)
    return (s << sh[None, :]).sum(axis=1).astype(np.uint8).tobytes()


def encrypt(data: bytes, B, nb: int, iv: int) -> np.ndarray:
    """CBC over n-bit segments with the table A = B^-1; iv in [0, 2^n)."""
    if not 0 <= int(iv) < (1 << nb) or len(B) != (1 << nb):
        raise ValueError("iv and the table must be n-bit: iv in [0, %d), %d entries"
                         % (1 << nb, 1 << nb))
    A = np.argsort(np.asarray(B))
    p = to_segments(data, nb)
    c = np.empty_like(p)
    prev = int(iv)
    for i, x in enumerate(p):
        prev = int(A[x ^ prev])
        c[i] = prev
    return c


def decrypt_with_codes(cipher, codes, nb: int, iv: int) -> bytes:
    """p_i = code_i xor c_{i-1}, where code_i is the bank's response to the
    key pair c_i selects."""
    if not 0 <= int(iv) < (1 << nb):
        raise ValueError("iv must be in [0, %d)" % (1 << nb))
    c = np.asarray(cipher, np.int64)
    prev = np.concatenate([[int(iv)], c[:-1]])
    return from_segments(np.asarray(codes, np.int64) ^ prev, nb)


def decrypt(cipher, key_f, key_A, model: dict, taus, nb: int, iv: int, T: int, window: int,
            dev: str = "cuda", timing: dict | None = None) -> bytes:
    """Decryption by simulation: the filter bank runs on the key pair of
    every ciphertext segment (one population of len(cipher) x n neurons)."""
    c = np.asarray(cipher, np.int64)
    codes = codes_from_levels(bank_levels(model, taus, np.asarray(key_f)[c], np.asarray(key_A)[c],
                                          T, window, dev, timing))
    return decrypt_with_codes(c, codes, nb, iv)
