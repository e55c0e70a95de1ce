"""A first stage for the delayed-acceptance test that is not learned: the
bare Coulomb energy of the neighbours within the histogram range, written as
weights of the library's network, so that it runs through the same kernels
as a trained network and isolates what training buys.

With phi the two 64-bin neighbour histograms of a position (like-charged
neighbours in inputs 0..63, unlike-charged in 64..127; bin k covers
[k dr, (k+1) dr), dr = rc / 64), the surrogate is

    eps(phi) = sum_k (phi_like[k] - phi_unlike[k]) / r_k,   r_k = (k + 1/2) dr,

so that l_B (eps(phi(x~)) - eps(phi(x))) is Eq. (Delta E_ij) for a 1:1
electrolyte truncated at rc with the neighbours placed at their bin centres.
As network weights: the first layer passes the counts through (identity,
counts are non-negative integers below 256, exact in bfloat16); the second
layer forms u = sum_k c_k phi_k in hidden unit 0 and -u in unit 1; the last
layer returns relu(u) - relu(-u) = u (to the bfloat16 rounding of the
activations).  Antisymmetric in the move by construction, as every network
output difference is.
"""
from __future__ import annotations

import numpy as np

BINS, HID = 64, 128
IN = 2 * BINS
NPARAM = IN * HID + HID + HID * HID + HID + HID + 1


def _bf16(a):
    """Round to the nearest bfloat16 value (ties to even), through float."""
    f = np.asarray(a, np.float32).copy()
    b = f.view(np.uint32)
    b += np.uint32(0x7FFF) + ((b >> np.uint32(16)) & np.uint32(1))
    b &= np.uint32(0xFFFF0000)
    return b.view(np.float32).astype(np.float64)


def truncated_coulomb_params(rc: float = 4.0) -> np.ndarray:
    """Flat parameter vector [W1 (row = input), b1, W2 (row = input), b2, w3,
    b3] of the truncated-Coulomb surrogate for features of range rc."""
    dr = rc / BINS
    inv_r = 1.0 / ((np.arange(BINS) + 0.5) * dr)
    c = np.concatenate([inv_r, -inv_r])
    W1 = np.eye(IN, HID)
    W2 = np.zeros((HID, HID))
    W2[:IN, 0] = c
    W2[:IN, 1] = -c
    w3 = np.zeros(HID)
    w3[0], w3[1] = 1.0, -1.0
    p = np.concatenate([W1.ravel(), np.zeros(HID), W2.ravel(), np.zeros(HID), w3, [0.0]])
    assert p.size == NPARAM
    return _bf16(p)
