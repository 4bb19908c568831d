"""First-order dual numbers a + b*eps (eps^2 = 0) over numpy arrays.

Used by the oracle gradient: running the unchanged recursion on dual inputs
with b = 1 on one momentum component gives that partial derivative exactly
(forward mode).  Values and derivatives may be real or complex arrays.
"""
import numpy as np


class Dual:
    __slots__ = ("v", "d")
    __array_ufunc__ = None  # numpy arrays defer to the reflected operators below

    def __init__(self, v, d=None):
        self.v = v
        self.d = np.zeros_like(v) if d is None else d

    # arithmetic -----------------------------------------------------------
    def __add__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v + o.v, self.d + o.d)
        return Dual(self.v + o, self.d)

    __radd__ = __add__

    def __sub__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v - o.v, self.d - o.d)
        return Dual(self.v - o, self.d)

    def __rsub__(self, o):
        return Dual(o - self.v, -self.d)

    def __neg__(self):
        return Dual(-self.v, -self.d)

    def __mul__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v * o.v, self.d * o.v + self.v * o.d)
        return Dual(self.v * o, self.d * o)

    __rmul__ = __mul__

    def __truediv__(self, o):
        if isinstance(o, Dual):
            return Dual(self.v / o.v, (self.d * o.v - self.v * o.d) / (o.v * o.v))
        return Dual(self.v / o, self.d / o)

    def __rtruediv__(self, o):
        return Dual(o / self.v, -o * self.d / (self.v * self.v))

    def __pow__(self, x):
        """Real power (x a Python number): d(a^x) = x a^(x-1) da."""
        vx = self.v ** x
        return Dual(vx, x * self.v ** (x - 1) * self.d)

    def conj(self):
        return Dual(np.conj(self.v), np.conj(self.d))

    @property
    def real(self):
        return Dual(np.real(self.v), np.real(self.d))


def value(x):
    """Plain value of a number that may be dual."""
    return x.v if isinstance(x, Dual) else x


def conj(x):
    return x.conj() if isinstance(x, Dual) else np.conj(x)


def real(x):
    return x.real if isinstance(x, Dual) else np.real(x)
