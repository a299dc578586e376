"""Philox4x32-10 counter-based generator (oracle side).

The paper only says "rand(0, 1)" (Metropolis criterion, Methods).  The
random stream is Philox4x32 with 10 rounds as published by Salmon, Moraes,
Dror and Shaw ("Parallel random numbers: as easy as 1, 2, 3", SC'11): a
128-bit counter and a 64-bit key; each round multiplies words 0 and 2 by two
fixed 32-bit constants, mixes the high halves with the other words and the
key, and the key is bumped by two Weyl constants between rounds.

Stream layout (reading): key = (ligand id, seed); counter = (trajectory,
step, purpose, block), purpose 0 = initial pose (blocks of 4 DOFs), 1 = one
MC step (word 0 -> DOF index, word 1 -> new value, word 2 -> acceptance).
A u32 x becomes u = (x >> 8) * 2^-24, exactly representable in FP32.
"""
import numpy as np

MUL0 = 0xD2511F53
MUL1 = 0xCD9E8D57
WEYL0 = 0x9E3779B9
WEYL1 = 0xBB67AE85
M32 = 0xFFFFFFFF


def philox4x32_10(counter, key):
    """counter: 4 uint32 (scalars or equal-shape arrays); key: 2 uint32."""
    c = [np.asarray(v, np.uint64) & M32 for v in counter]
    k0 = np.asarray(key[0], np.uint64) & M32
    k1 = np.asarray(key[1], np.uint64) & M32
    for _ in range(10):
        p0 = np.uint64(MUL0) * c[0]
        p1 = np.uint64(MUL1) * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(M32)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(M32)
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(WEYL0)) & np.uint64(M32)
        k1 = (k1 + np.uint64(WEYL1)) & np.uint64(M32)
    return [v.astype(np.uint32) for v in c]


def to_unit(x):
    """u32 -> uniform in [0, 1) with 24 bits: (x >> 8) * 2^-24."""
    return (np.asarray(x, np.uint32) >> np.uint32(8)).astype(np.float64) * (2.0 ** -24)


def mulhi_index(x, n):
    """floor(x * n / 2^32): an index in [0, n) from a u32."""
    return ((np.asarray(x, np.uint64) * np.uint64(n)) >> np.uint64(32)).astype(np.int64)


PURPOSE_INIT = 0
PURPOSE_STEP = 1


def draw(lig, seed, traj, step, purpose, block=0):
    """One Philox call; traj may be an array.  Returns 4 uint32 arrays."""
    traj = np.asarray(traj, np.uint64)
    z = np.zeros_like(traj)
    return philox4x32_10([traj, z + np.uint64(step), z + np.uint64(purpose), z + np.uint64(block)],
                         [np.uint64(lig) + z, np.uint64(seed) + z])
