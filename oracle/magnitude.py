"""Magnitude numbers: a value together with the magnitude of its evaluation
(TEST INFRASTRUCTURE).

A ``Mag`` carries the value v of an expression and m, the same expression
evaluated with every input replaced by its modulus and every subtraction by
an addition (for a quotient the divisor is taken as an exact input).  For a
computation built from additions and multiplications, a floating-point
evaluation with unit roundoff u in which every input and every operation is
rounded once differs from the exact value by at most about (depth) u m
(the classical running error bound); m / |v| is therefore the condition
number of the value with respect to such rounding.  Running the unchanged
colour-ordered recursion (Section 2.3) and the colour sum (Section 2.2) on
magnitude numbers gives, per event, the scale against which the rounding
error of any evaluation order is judged: the floating-point tolerances of the
tests are stated as multiples of u m.
"""
import numpy as np


class Mag:
    __slots__ = ("v", "m")
    __array_ufunc__ = None  # numpy arrays defer to the reflected operators below

    def __init__(self, v, m=None):
        self.v = v
        self.m = np.abs(v) if m is None else m

    def __add__(self, o):
        if isinstance(o, Mag):
            return Mag(self.v + o.v, self.m + o.m)
        return Mag(self.v + o, self.m + np.abs(o))

    __radd__ = __add__

    def __sub__(self, o):
        if isinstance(o, Mag):
            return Mag(self.v - o.v, self.m + o.m)
        return Mag(self.v - o, self.m + np.abs(o))

    def __rsub__(self, o):
        return Mag(o - self.v, np.abs(o) + self.m)

    def __neg__(self):
        return Mag(-self.v, self.m)

    def __mul__(self, o):
        if isinstance(o, Mag):
            return Mag(self.v * o.v, self.m * o.m)
        return Mag(self.v * o, self.m * np.abs(o))

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Mag):
            return Mag(self.v / o.v, self.m / np.abs(o.v))
        return Mag(self.v / o, self.m / np.abs(o))

    def __rtruediv__(self, o):
        return Mag(o / self.v, np.abs(o) / np.abs(self.v))


def lift(vec):
    """A four-vector of plain arrays -> four-vector of magnitude numbers."""
    return [Mag(c) for c in vec]
