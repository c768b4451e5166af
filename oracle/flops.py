"""A counting number type for FLOP pins (oracle; test infrastructure only).

The paper counts operations with the Livermore convention (Sec. 2.5): addition,
subtraction and multiplication cost 1 FLOP, division 4. Negation is free.
Running one of the scalar oracle solvers on ``Flop`` values counts exactly the
operations that its source performs.
"""
from __future__ import annotations


class Counter:
    def __init__(self):
        self.add = 0
        self.mul = 0
        self.div = 0

    @property
    def flops(self):
        return self.add + self.mul + 4 * self.div


class Flop:
    """A float that charges every arithmetic operation to a shared Counter."""

    __slots__ = ("v", "c")

    def __init__(self, v, c):
        self.v = float(v)
        self.c = c

    def _val(self, o):
        return o.v if isinstance(o, Flop) else float(o)

    def __add__(self, o):
        self.c.add += 1
        return Flop(self.v + self._val(o), self.c)

    __radd__ = __add__

    def __sub__(self, o):
        self.c.add += 1
        return Flop(self.v - self._val(o), self.c)

    def __rsub__(self, o):
        self.c.add += 1
        return Flop(self._val(o) - self.v, self.c)

    def __mul__(self, o):
        self.c.mul += 1
        return Flop(self.v * self._val(o), self.c)

    __rmul__ = __mul__

    def __truediv__(self, o):
        self.c.div += 1
        return Flop(self.v / self._val(o), self.c)

    def __rtruediv__(self, o):
        self.c.div += 1
        return Flop(self._val(o) / self.v, self.c)

    def __neg__(self):
        return Flop(-self.v, self.c)

    def __float__(self):
        return self.v


def count(fn, *numeric_args, **kw):
    """Run ``fn`` with every number in ``numeric_args`` (scalars or flat
    sequences) wrapped as Flop; return (result, Counter)."""
    c = Counter()

    def wrap(a):
        if isinstance(a, (list, tuple)):
            return [Flop(x, c) for x in a]
        return Flop(a, c)

    out = fn(*[wrap(a) for a in numeric_args], **kw)
    return out, c
