"""A slot simulator with the oracle evaluator's interface, on plain FP64 arrays.

TEST INFRASTRUCTURE ONLY.  A "ciphertext" here is (level, slot vector): add
is +, ct x ct is *, rotation by t is a left cyclic shift (np.roll(v, -t)),
plaintext products are elementwise.  Levels move exactly as in the oracle's
RNS-CKKS evaluator, so running the circuit on this class checks the circuit's
logic (packing, rotation amounts, diagonal layout, polynomial splitting and
the level plan) against plain linear algebra, with no encryption involved.
"""
from dataclasses import dataclass

import numpy as np


@dataclass
class SimCt:
    level: int
    v: np.ndarray


class _P:
    def __init__(self, slots):
        self.slots = slots


class _Ctx:
    def __init__(self, slots):
        self.p = _P(slots)


class SlotSim:
    def __init__(self, slots):
        self.ctx = _Ctx(slots)
        self.count = {"ks": 0, "rescale": 0, "rot": 0}
        self.rot_steps = set()

    def fresh(self, z, level):
        v = np.zeros(self.ctx.p.slots)
        v[: len(z)] = z
        return SimCt(level, v)

    def add(self, a, b):
        assert a.level == b.level
        return SimCt(a.level, a.v + b.v)

    def sub(self, a, b):
        assert a.level == b.level
        return SimCt(a.level, a.v - b.v)

    def mul_int(self, a, k):
        return SimCt(a.level, a.v * k)

    def add_const(self, a, c):
        return SimCt(a.level, a.v + c)

    def add_vec(self, a, z):
        return SimCt(a.level, a.v + np.asarray(z))

    def mod_drop(self, a, l):
        assert l <= a.level
        return SimCt(l, a.v)

    def tensor(self, a, b):
        assert a.level == b.level
        return [a.level, a.v * b.v]

    def tensor_add(self, t1, t2):
        assert t1[0] == t2[0]
        return [t1[0], t1[1] + t2[1]]

    def relin_rescale(self, t):
        self.count["ks"] += 1
        self.count["rescale"] += 1
        assert t[0] >= 1
        return SimCt(t[0] - 1, t[1])

    def mul(self, a, b):
        return self.relin_rescale(self.tensor(a, b))

    def rotate(self, a, t):
        if t % self.ctx.p.slots == 0:
            return a
        self.count["ks"] += 1
        self.count["rot"] += 1
        self.rot_steps.add(t)
        return SimCt(a.level, np.roll(a.v, -t))

    def rotate_sum(self, items):
        """sum_i rot(x_i, t_i), the rotations sharing one ModDown (no
        difference on plain vectors)."""
        level = items[0][0].level
        acc = np.zeros(self.ctx.p.slots)
        for x, t in items:
            assert x.level == level
            acc = acc + self.rotate(x, t).v
        return SimCt(level, acc)

    def lincomb(self, terms, t):
        acc = np.zeros(self.ctx.p.slots)
        for ct, z in terms:
            assert ct.level >= t + 1, (ct.level, t)
            acc = acc + ct.v * z
        assert t >= 0
        self.count["rescale"] += 1
        return SimCt(t, acc)

    def level_down(self, a, t):
        if a.level == t:
            return a
        assert a.level > t
        return self.lincomb([(a, 1.0)], t)
