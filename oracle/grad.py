"""Adjoints of the projected product and of the projection, float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper defines the forward maps only; the gradients follow from Def. 3.1
by the chain rule.  Writing C_(3) = Q Ch_(3), Ch = Ah tri Bh,
Ah_(3) = Q^T A_(3), Bh_(3) = Q^T B_(3) and G = dL/dC:

    dCh    = G x_3 Q^T
    dAh_l  = dCh_l Bh_l^T          dBh_l = Ah_l^T dCh_l      (each face l)
    dA     = dAh x_3 Q             dB    = dBh x_3 Q
    dQ     = G_(3) Ch_(3)^T + A_(3) dAh_(3)^T + B_(3) dBh_(3)^T

(the Euclidean gradient of Q treated as a free n3 x p matrix).  For
P = A x_3 Q Q^T:  dA = G x_3 Q Q^T and dQ = G_(3) A_(3)^T Q + A_(3) G_(3)^T Q.
"""

import numpy as np

from .core import hat, unhat, facewise, unfold3, _f64


def qprod_backward(G, A, B, Q):
    G, A, B, Q = _f64(G), _f64(A), _f64(B), _f64(Q)
    Ah, Bh = hat(A, Q), hat(B, Q)
    Ch = facewise(Ah, Bh)
    dCh = hat(G, Q)
    dAh = facewise(dCh, np.transpose(Bh, (1, 0, 2)))
    dBh = facewise(np.transpose(Ah, (1, 0, 2)), dCh)
    dA = unhat(dAh, Q)
    dB = unhat(dBh, Q)
    dQ = (unfold3(G) @ unfold3(Ch).T
          + unfold3(A) @ unfold3(dAh).T
          + unfold3(B) @ unfold3(dBh).T)
    return dA, dB, dQ


def proj_backward(G, A, Q):
    G, A, Q = _f64(G), _f64(A), _f64(Q)
    dA = unhat(hat(G, Q), Q)
    G3, A3 = unfold3(G), unfold3(A)
    dQ = G3 @ (A3.T @ Q) + A3 @ (G3.T @ Q)
    return dA, dQ
