"""Working precision of the oracle (TEST INFRASTRUCTURE).

Every oracle function computes in the precision of its inputs: float64
momenta give the plain FP64 oracle, ``np.longdouble`` momenta (x87 80-bit,
64-bit significand, unit roundoff 5.4e-20) give the extended reference the
floating-point bars of the tests are measured against, and numpy object
arrays of ``mpmath.mpf`` give an arbitrary-precision evaluation that pins the
extended one.  The irrational constants of the paper (sqrt 2 in the vertices
and polarizations of Sections 2.1 and 2.3, g_s = sqrt(4 pi alpha_s) with
alpha_s = 0.118 of Section 5) are formed here in that same precision, so an
extended evaluation is not limited by a constant rounded to FP64.
"""
import math

import numpy as np

ALPHA_S_TEXT = "0.118"
PI_TEXT = "3.14159265358979323846264338327950288419716939937510"


def _leaf(x):
    """A representative scalar or array of x (unwraps dual and magnitude numbers)."""
    while hasattr(x, "v") and not isinstance(x, np.ndarray):
        x = x.v
    return x


def kind(like):
    """'f64', 'ld' (long double) or 'mp' (mpmath objects) for a value or array."""
    x = _leaf(like)
    if isinstance(x, (list, tuple)):
        return kind(x[0])
    dt = getattr(x, "dtype", None)
    if dt is not None:
        if dt in (np.longdouble, np.clongdouble):
            return "ld"
        if dt == object:
            flat = np.ravel(x)
            return kind(flat[0]) if flat.size else "f64"
        return "f64"
    if isinstance(x, (np.longdouble, np.clongdouble)):
        return "ld"
    if type(x).__module__.startswith("mpmath"):
        return "mp"
    return "f64"


def sqrt2(like):
    """sqrt(2) in the precision of `like`."""
    k = kind(like)
    if k == "ld":
        return np.sqrt(np.longdouble(2))
    if k == "mp":
        import mpmath
        return mpmath.sqrt(2)
    return math.sqrt(2.0)


def coupling(like):
    """g_s = sqrt(4 pi alpha_s) in the precision of `like`."""
    k = kind(like)
    if k == "ld":
        return np.sqrt(np.longdouble(4) * np.longdouble(PI_TEXT) * np.longdouble(ALPHA_S_TEXT))
    if k == "mp":
        import mpmath
        return mpmath.sqrt(4 * mpmath.pi * mpmath.mpf(ALPHA_S_TEXT))
    return math.sqrt(4.0 * math.pi * float(ALPHA_S_TEXT))


def complex_type(like):
    """The complex dtype matching `like` (object for mpmath arrays)."""
    k = kind(like)
    return {"ld": np.clongdouble, "mp": object}.get(k, np.complex128)


def extended(a):
    """Convert a float64 array to the extended (long double) working precision."""
    return np.asarray(a, dtype=np.float64).astype(np.longdouble)


def arbitrary(a, dps=40):
    """Convert a float64 array to mpmath numbers with `dps` decimal digits (object array)."""
    import mpmath
    mpmath.mp.dps = dps
    return np.vectorize(lambda x: mpmath.mpf(float(x)), otypes=[object])(np.asarray(a))
