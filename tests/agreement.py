"""Agreement of two converged PageRank results of the same graph (say, one
update run alone and the same update run among many graphs).

Both stop when no rank changes by more than tol in a sweep.  The error left
at that point lies mostly along the slowest-decaying direction of the
iteration: the total rank mass, which Eq. 1 moves toward 1 by a factor alpha
per sweep (its error vector is proportional to the ranks themselves), while
the other directions decay at least as fast.  A change below tol in every
rank leaves up to about tol * alpha / (1 - alpha) (5.7e-10 at the paper's
tol 1e-10, alpha 0.85) along it, with a sign that depends on the order the
vertices were processed in.  Two results that are each within the bar of
the fixed point can therefore differ by up to twice the bar, and only along
that direction.  `agree` checks exactly that: the difference with its
mass-direction part removed is within the bar, and the whole difference
within twice the bar."""
import numpy as np


def agree(a, b, ref, bar, relative=False):
    """a, b: the two results; ref: the oracle's fixed point (the direction
    of the mass error); bar: L-infinity bar, relative to max|ref| when
    `relative`.  Returns (ok, orthogonal part, whole difference), both
    difference norms in the bar's units."""
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    ref = np.asarray(ref, np.float64)
    d = a - b
    mu = d.sum() / ref.sum()
    scale = float(np.abs(ref).max()) if relative else 1.0
    perp = float(np.abs(d - mu * ref).max()) / scale
    whole = float(np.abs(d).max()) / scale
    return perp <= bar and whole <= 2 * bar, perp, whole
