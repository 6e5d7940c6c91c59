"""Slot-level simulator of the CKKS operations (complex128 vectors, exact up to FP64).

TEST INFRASTRUCTURE ONLY.  A ciphertext is modelled by its slot vector and its
level; rotation is a cyclic shift of the vector (Sec. 2.2: Lrot(ct, r) moves
slot r to slot 0), conjugation is slot-wise, multiplications are slot-wise and
the level bookkeeping mirrors the encrypted evaluator's (mult and cmult are
followed by an explicit rescale that consumes one level).  It runs the matrix
algorithms at the paper's shapes in milliseconds and counts their operations.
"""
import numpy as np

from .ckks import LevelError


class SimCt:
    def __init__(self, z, level):
        self.z = np.asarray(z, dtype=np.complex128)
        self.level = int(level)
        self.scale = 1.0


class SimEvaluator:
    def __init__(self, slots):
        self.slots = slots
        self.counts = {}

    def _count(self, name, k=1):
        self.counts[name] = self.counts.get(name, 0) + k

    def reset_counts(self):
        self.counts = {}

    @staticmethod
    def level(ct):
        return ct.level

    def encrypt(self, z, level):
        z = np.asarray(z, dtype=np.complex128)
        assert z.shape == (self.slots,)
        return SimCt(z.copy(), level)

    def decrypt(self, ct):
        return ct.z.copy()

    def add(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch %d vs %d" % (a.level, b.level))
        return SimCt(a.z + b.z, a.level)

    def sub(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch %d vs %d" % (a.level, b.level))
        return SimCt(a.z - b.z, a.level)

    def mul_i(self, a):
        return SimCt(1j * a.z, a.level)

    def mod_drop(self, a, level):
        if level > a.level or level < 0:
            raise LevelError("cannot drop level %d to %d" % (a.level, level))
        return SimCt(a.z.copy(), level)

    def rescale(self, a):
        if a.level < 1:
            raise LevelError("no level left to rescale")
        self._count("rescale")
        return SimCt(a.z.copy(), a.level - 1)

    def cmult_mask(self, a, values):
        self._count("cmult")
        return SimCt(a.z * np.asarray(values, dtype=np.complex128), a.level)

    def mult(self, a, b):
        if a.level != b.level:
            raise ValueError("level mismatch")
        self._count("mult")
        self._count("keyswitch")
        return SimCt(a.z * b.z, a.level)

    def rot(self, a, r):
        self._count("rot")
        self._count("keyswitch")
        return SimCt(np.roll(a.z, -r), a.level)

    def conj(self, a):
        self._count("conj")
        self._count("keyswitch")
        return SimCt(np.conj(a.z), a.level)
