"""Second-order jets of two variables for manufactured solutions (test helper).

A Jet carries a field's value, gradient (d/dx, d/dy) and Hessian (xx, xy, yy)
as NumPy arrays, closed under +, -, *, scalar operations and sin/cos/exp by
the product and chain rules, so continuous operators of closed-form fields
(here the stress divergence of an isotropic medium with variable Lame
parameters) are evaluated exactly, without a symbolic package.
"""

import numpy as np


class Jet:
    def __init__(self, v, gx, gy, hxx, hxy, hyy):
        self.v, self.gx, self.gy = v, gx, gy
        self.hxx, self.hxy, self.hyy = hxx, hxy, hyy

    @staticmethod
    def var_x(x):
        z = np.zeros_like(x)
        return Jet(x, np.ones_like(x), z, z, z, z)

    @staticmethod
    def var_y(y):
        z = np.zeros_like(y)
        return Jet(y, z, np.ones_like(y), z, z, z)

    @staticmethod
    def const(c, like):
        z = np.zeros_like(like)
        return Jet(np.full_like(like, c), z, z, z, z, z)

    def _lift(self, o):
        return o if isinstance(o, Jet) else Jet.const(float(o), self.v)

    def __add__(self, o):
        o = self._lift(o)
        return Jet(self.v + o.v, self.gx + o.gx, self.gy + o.gy, self.hxx + o.hxx, self.hxy + o.hxy, self.hyy + o.hyy)

    __radd__ = __add__

    def __neg__(self):
        return Jet(-self.v, -self.gx, -self.gy, -self.hxx, -self.hxy, -self.hyy)

    def __sub__(self, o):
        return self + (-self._lift(o))

    def __rsub__(self, o):
        return self._lift(o) - self

    def __mul__(self, o):
        o = self._lift(o)
        return Jet(self.v * o.v,
                   self.gx * o.v + self.v * o.gx,
                   self.gy * o.v + self.v * o.gy,
                   self.hxx * o.v + 2 * self.gx * o.gx + self.v * o.hxx,
                   self.hxy * o.v + self.gx * o.gy + self.gy * o.gx + self.v * o.hxy,
                   self.hyy * o.v + 2 * self.gy * o.gy + self.v * o.hyy)

    __rmul__ = __mul__

    def _chain(self, f0, f1, f2):
        """g(self) with g = f0, g' = f1, g'' = f2 evaluated at self.v."""
        return Jet(f0, f1 * self.gx, f1 * self.gy,
                   f2 * self.gx * self.gx + f1 * self.hxx,
                   f2 * self.gx * self.gy + f1 * self.hxy,
                   f2 * self.gy * self.gy + f1 * self.hyy)


def sin(a):
    return a._chain(np.sin(a.v), np.cos(a.v), -np.sin(a.v))


def cos(a):
    return a._chain(np.cos(a.v), -np.sin(a.v), -np.cos(a.v))


def exp(a):
    e = np.exp(a.v)
    return a._chain(e, e, e)


def stress_divergence(u, v, lam, mu):
    """div s for s = lam (div U) I + mu (grad U + grad U^T), U = (u, v) jets,
    lam and mu jets (their first derivatives are used).  Returns two arrays."""
    div = u.gx + v.gy
    div_x = u.hxx + v.hxy
    div_y = u.hxy + v.hyy
    shear = u.gy + v.gx
    fx = (lam.gx * div + lam.v * div_x + 2 * mu.gx * u.gx + 2 * mu.v * u.hxx
          + mu.gy * shear + mu.v * (u.hyy + v.hxy))
    fy = (mu.gx * shear + mu.v * (u.hxy + v.hxx) + lam.gy * div + lam.v * div_y
          + 2 * mu.gy * v.gy + 2 * mu.v * v.hyy)
    return fx, fy
