"""Pins of the oracle's operation counter (the roofline's algorithmic flops).

Counting rule of the counting scalar: +, -, *, / and sqrt each count one;
an operation counts unless it is trivial -- a product with an exact 0, +1 or
-1 operand, a sum or difference with an exact 0 operand, a division of an
exact 0 or by +-1.  Negation and copies are free.  sin, cos, atan2 and log
are counted apart (column 4).  Columns: add/sub, mul, div, sqrt, trans.

The expected counts below are derived by hand from the textbook operation
sequence of each step (dense where the inputs are dense, with the structural
zeros and ones the step itself creates), not read off the counter.  "Generic"
inputs have no entry equal to 0 or +-1, so the only trivial operations are
the structural ones named in each derivation.

The whole-track check then shows that the count of a whole fit is exactly the
sum of these pinned units applied to the track's own states: nothing else in
the fit is counted.
"""
import math

import numpy as np
import pytest

import oracle
from paper_2105_01796_amd import synth

ADD, MUL, DIV, SQRT, TRANS = range(5)


def _spd(rng, n=6):
    a = rng.standard_normal((n, n))
    return a @ a.T + n * np.eye(n)


def _tilted_pair():
    """Two generic planes (every centre and rotation entry nonzero, none +-1)."""
    det = synth.telescope(2, x_over_X0=0.005)
    al = np.array([[0.9, -3.2, 4.1, 0.11, -0.23, 0.31],
                   [2.3, 1.7, -5.1, -0.17, 0.29, 0.05],
                   [0.0, 0.0, 0.0, 0.0, 0.0, 0.0]]).T
    det = synth.misalign(det, al)
    assert np.all(det.center[:, :2] != 0.0) and np.all(np.abs(det.rot[:, :2]) != 1.0)
    assert np.all(det.rot[:, :2] != 0.0)
    return det


def _unit_norm(phi, theta):
    """Whether the bound->free direction (cos phi sin theta, sin phi sin theta,
    cos theta) has |T|^2 == 1 exactly in FP64.  Python's math module calls the
    same C library sin/cos as the oracle, which is built without FMA
    contraction, so this reproduces the oracle's rounding."""
    tx, ty, tz = math.cos(phi) * math.sin(theta), math.sin(phi) * math.sin(theta), math.cos(theta)
    return (tx * tx + ty * ty) + tz * tz == 1.0


def test_count_gain_update_dense():
    """One update with H = [I2 0], dense generic Cp (6x6), V (v01 != 0), m, xp.
      r = m - H xp                         2 add
      S = V + H Cp H^T (4 entries)         4 add
      det S                                2 mul, 1 add
      S^-1 (4 entries / det)               4 div
      K = Cp H^T S^-1 (6x2, 2 terms each)  24 mul, 12 add
      xf = xp + K r (6 x 2 terms)          12 mul, 12 add
      I - K H: only the diagonal 1 - K_ii (i < 2) is nontrivial: 2 add
      (I-KH) Cp: per entry k = 0, 1 nontrivial (2 mul); the identity column
        k = i (i >= 2) adds a third term: adds 1 (i < 2) or 2 (i >= 2),
        36 entries: 72 mul, 6 * (2*1 + 4*2) = 60 add
      ((I-KH) Cp) (I-KH)^T: the same pattern by column: 72 mul, 60 add
      K V K^T: per entry 4 terms of 2 mul, 3 add, + the Joseph sum 1 add:
        36 * (8 mul, 4 add) = 288 mul, 144 add
      chi2 = r^T S^-1 r                    6 mul, 3 add
    Total: add 2+4+1+12+12+2+60+60+144+3 = 300, mul 2+24+12+72+72+288+6 = 476,
    div 4."""
    rng = np.random.default_rng(6)
    st, c = oracle.count_update(0.1 * rng.standard_normal(6), _spd(rng), 0.1 * rng.standard_normal(2),
                                [0.3, 0.1, 0.4])
    assert st == 0
    assert c.tolist() == [300, 476, 4, 0, 0]


def test_count_rts_step_dense():
    """One RTS step, dense generic Cf, F, Cp1, Cs1 (6x6) and vectors.
      Cholesky of Cp1: column j has j mul/add for the pivot, 1 sqrt, and for
        each of the 5-j rows below j mul/add and 1 div:
        mul = add = sum_j (j + (5-j) j) = 35, sqrt 6, div 5+4+3+2+1 = 15
      F Cf (6x6x6): 216 mul, 6*6*5 = 180 add
      solve (L L^T) A^T = F Cf, 6 right-hand sides, each forward + backward:
        2 * (15 mul, 15 add, 6 div) -> 6 * (30 mul, 30 add, 12 div)
        = 180 mul, 180 add, 72 div
      dx = xs1 - xp1                       6 add
      xs = xf + A dx (acc starts at xf)    36 mul, 36 add
      dC = Cs1 - Cp1                       36 add
      A dC, (A dC) A^T                     2 * (216 mul, 180 add)
      Cs = Cf + ...                        36 add
    Total: mul 35+216+180+36+432 = 899, add 35+180+180+6+36+36+360+36 = 869,
    div 15+72 = 87, sqrt 6.  (States with phi differences within (-pi, pi]:
    a wrap by 2 pi would add one more operation.)"""
    rng = np.random.default_rng(6)
    st, c = oracle.count_rts_step(0.1 * rng.standard_normal(6), _spd(rng), rng.standard_normal((6, 6)),
                                  0.1 * rng.standard_normal(6), _spd(rng), 0.1 * rng.standard_normal(6), _spd(rng))
    assert st == 0
    assert c.tolist() == [869, 899, 87, 6, 0]


def test_count_field_free_transport_without_step():
    """Field off, generic tilted planes a -> b, landing tolerance above the
    distance, so the propagation takes no RKN trial and the final second-order
    move covers the whole distance.
      bound -> free: 4 trig; r = c + l0 u + l1 v (3 x (2 mul, 2 add));
        T = (cp st, sp st, ct) 2 mul; J columns -sp st, cp st, cp ct, sp ct
        4 mul                                      12 mul, 6 add, 4 trans
      loop test: n.T (3 mul, 2 add); n.(c - r) (3 add, 3 mul, 2 add)
                                                   6 mul, 7 add
      final move: n.T, n.(c - r) again (6 mul, 7 add), d = dist/n.T (1 div);
        B = 0 makes T x B = 0: r_i += d T_i + (((0.5 d) d) lam) kB (T x B)_i
        5 mul + 1 add each (the product with 0 and the sum with 0 are free);
        T_i += ((d lam) kB) (T x B)_i 2 mul each; t += d sqrt(1 + m^2 lam^2)/c
        (m^2 is a constant: lam * (m^2) and * lam 2 mul, 1 add, 1 sqrt,
        d * 1 mul, / c 1 div, t + 1 add)       30 mul, 12 add, 2 div, 1 sqrt
      path correction: dF/ds: lam kB (3 mul, times 0 free), dt/ds (2 mul,
        1 add, 1 sqrt, 1 div); n.T (3 mul, 2 add); P = I - dF/ds n^T / n.T:
        nonzero for rows r, t (4) x columns r (3): 12 mul, 12 div, and the
        3 diagonal entries 1 - x: 3 add         20 mul, 6 add, 13 div, 1 sqrt
      free -> bound: r - c 3 add; u.d, v.d 6 mul, 4 add; rho^2 2 mul, 1 add;
        rho 1 sqrt; n2 = rho^2 + tz^2 1 mul, 1 add; 2 atan2; J rows: -ty/rho^2,
        tx/rho^2 2 div; tx tz/(rho n2), ty tz/(rho n2) 4 mul, 2 div;
        -rho/n2 1 div                            13 mul, 9 add, 5 div, 1 sqrt, 2 trans
      J_fb P (6x8 x 8x8): rows loc0, loc1 see P's generic 3x3 block: 2 x 3
        entries x (3 mul, 2 add); every other product hits 0 or 1
                                                   18 mul, 12 add
      (J_fb P) D with D = I (no step): 0
      ((J_fb P) D) J_bf (6x8 x 8x6): rows loc0, loc1, t x columns loc0, loc1:
        6 x (3 mul, 2 add); row phi: 2 x (2 mul, 1 add); row theta:
        (2 mul, 1 add) + (3 mul, 2 add)           27 mul, 17 add
    Total: mul 12+6+30+20+13+18+27 = 126, add 6+7+12+6+9+12+17 = 69,
    div 2+13+5 = 20, sqrt 3, trans 6.
    When |T|^2 is exactly 1 in FP64, n2 = 1 makes rho * n2 (twice) and
    -rho / n2 trivial: mul 124, div 19."""
    det = _tilted_pair()
    fld0 = synth.Field(0, (0.0, 0.0, 0.0), 0.0)
    seen = set()
    for phi, theta in [(-0.09, 1.43), (0.05, 1.55), (0.07, 1.52), (0.11, 1.47)]:
        x = np.array([1.3, -2.1, phi, theta, 0.37, 0.8])
        st, c, trials = oracle.count_transport(det, fld0, 0, 1, x, land_tol=1e3)
        assert st == 0 and trials == 0
        unit = _unit_norm(phi, theta)
        seen.add(unit)
        expect = [69, 124, 19, 3, 6] if unit else [69, 126, 20, 3, 6]
        assert c.tolist() == expect, (phi, theta, unit)
    assert seen == {True, False}


def test_count_field_free_transport_one_step():
    """The same transport with the usual landing tolerance: one RKN trial of
    length h = d, accepted, then the landing test passes.  On top of the
    no-step count (generic |T|^2):
      first trial size d = dist / n.T            1 div
      RKN step with B = 0 (every stage k = lam kB (T x B) = 0):
        h/2, h^2                                  2 mul
        4 stages: k (lam kB: 3 mul) and dk (lam kB for each of the 24
          entries: 24 mul, times 0 free)          4 x 27 = 108 mul
        midpoint and end point: r + h' T (2 mul, 1 add) per axis and the
          hh/8 (hh/2) factor of each of the 24 dr entries
                                                  2 x (30 mul, 3 add)
        new state: r + h T (1 mul, 1 add) + hh/6 (1 div) per axis, h/6 per
          direction axis (1 div); sqrt(1 + m^2 lam^2) (2 mul, 1 add, 1 sqrt);
          t + h g / c (1 mul, 1 div, 1 add)        6 mul, 5 add, 7 div, 1 sqrt
        D: hh/6 and h/6 per entry of the 24 + 24 position/direction entries
          (48 div; the stage sums are 0); D_t,lam = h m m lam / (c g) (4 mul,
          1 div)                                   4 mul, 49 div
        step total 180 mul, 11 add, 56 div, 1 sqrt
      D_step D with D = I: 0
      second loop test                            6 mul, 7 add
      J_fb P D: D = I + h at (r_i, T_i) + D_t,lam: rows loc0, loc1, t pick
        up A_{r,i} h in the three direction columns   9 mul
      ... J_bf: rows loc0, loc1, t gain the phi/theta columns (2 mul + 1 add,
        3 mul + 2 add each)                        42 - 27 = 15 mul, 26 - 17 = 9 add
    Total: add 69+11+7+9 = 96, mul 126+180+6+9+15 = 336, div 20+1+56 = 77,
    sqrt 3+1 = 4, trans 6.  If the landing remainder rounds to exactly 0, the
    final move's d-terms are free: add 92, mul 314, div 75."""
    det = _tilted_pair()
    fld0 = synth.Field(0, (0.0, 0.0, 0.0), 0.0)
    x = np.array([1.3, -2.1, -0.09, 1.43, 0.37, 0.8])
    assert not _unit_norm(-0.09, 1.43)
    st, c, trials = oracle.count_transport(det, fld0, 0, 1, x, land_tol=1e-6)
    assert st == 0 and trials == 1
    assert c.tolist() in ([96, 336, 77, 4, 6], [92, 314, 75, 4, 6])


def test_count_rkn_step_uniform_field():
    """One RKN step (free state and its 8x8 Jacobian at fixed h) in a generic
    uniform field (every B component nonzero, none +-1; dB/dr = 0).
      h/2, h^2                                    2 mul
      stage 1 (dT = [0 | I3 | 0]): T x B 6 mul 3 add; k = (lam kB) (T x B)
        6 mul; dk: lam kB per entry (24 mul), times c1 where c1 = e_j x B has
        2 nonzero entries (columns T: 3 x 2 mul), column q/p + kB (T x B)
        (3 mul)                                   45 mul, 3 add
      midpoint r2, T2 (3 x (4 mul, 3 add)); dr2: hh/8 per entry (24 mul) and
        hh/8 dk1 on dk1's 9 nonzero entries (9 mul); dT2 = dT1 + h/2 dk1
        (9 mul; dT1's ones sit where dk1 = 0)      54 mul, 9 add
      stage 2 (dT columns T: one exact 1 each): T2 x B 6 mul 3 add; k 6 mul;
        columns loc/t 12 mul; columns T 3 x (4 mul, 3 add + 6 mul);
        column q/p 6 mul 3 add + 6 mul + 3 mul 3 add   69 mul, 18 add
      T3 (3 mul, 3 add); dT3 = dT1 + h/2 dk2 (12 mul, 3 add)   15 mul, 6 add
      stage 3 (dT columns T, q/p generic): 6+6+12+3x12+15 = 75 mul,
        3+3x3+6 = 18 add
      end point r4, T4 (3 x (4 mul, 3 add)); dr4 (24 + 12 mul, 3 add);
        dT4 (12 mul, 3 add)                       60 mul, 15 add
      stage 4 as stage 3                          75 mul, 18 add
      new state: r (2 mul, 4 add, 1 div per axis), T (3 mul, 4 add, 1 div),
        g (2 mul, 1 add, 1 sqrt), t (1 mul, 1 add, 1 div)
                                                  18 mul, 26 add, 7 div, 1 sqrt
      D position rows: hh/6 per entry (24 div); columns T and q/p:
        2 add, 1 mul each (12 entries)            12 mul, 24 add, 24 div
      D direction rows: h/6 per entry (24 div); 12 entries x (3 mul, 3 add)
                                                  36 mul, 36 add, 24 div
      D_t,lam = h m m lam / (c g)                 4 mul, 1 div
    Total: mul 465, add 173, div 56, sqrt 1."""
    fld = synth.Field(0, (0.3, -0.7, 2.0), 0.0)
    T = np.array([0.8, 0.3, 0.5])
    T /= np.linalg.norm(T)
    F = np.array([10.0, -3.0, 7.0, 0.4, *T, 0.37])
    assert oracle.count_rkn_step(fld, F, 23.7).tolist() == [173, 465, 56, 1, 0]


def test_count_scatterer_noise():
    """Highland noise on a generic tilted plane:
      st, T = (cos phi st, sin phi st, cos theta): 4 trig, 2 mul
      n.T 3 mul 2 add; path = x/X0 / |n.T| 1 div; p = 1/|q/p| 1 div;
      beta = p / sqrt(p^2 + m^2): 1 mul, 1 add, 1 sqrt, 1 div;
      theta0 = 0.0136/(beta p) sqrt(path) (1 + 0.038 log(path/beta^2)):
        beta p, *sqrt, beta^2, 0.038 *, * (1 + ...) 5 mul; 2 div; 1 sqrt;
        1 add; log
      Q22 = theta0^2 / st^2 (2 mul, 1 div); Q33 = theta0^2 (1 mul)
    Total: add 4, mul 14, div 6, sqrt 2, trans 5."""
    det = _tilted_pair()
    x = np.array([1.3, -2.1, -0.09, 1.43, 0.37, 0.8])
    assert oracle.count_ms_noise(det, 1, x).tolist() == [4, 14, 6, 2, 5]


def test_count_covariance_prediction_dense():
    """F (C + Q) F^T with dense generic F and C and Q = diag(0, 0, q22, q33, 0, 0):
    C + Q 2 add; two dense 6x6x6 products 2 x (216 mul, 180 add).
    Total: add 362, mul 432."""
    rng = np.random.default_rng(6)
    Q = np.zeros((6, 6))
    Q[2, 2], Q[3, 3] = 1e-6, 2e-6
    assert oracle.count_cov_transport(rng.standard_normal((6, 6)), _spd(rng), Q).tolist() == [362, 432, 0, 0, 0]


@pytest.mark.parametrize("cfg", [1, 2, 3, 5, 6, 7])
def test_count_whole_track_is_the_sum_of_units(cfg):
    """The count of a whole fit equals, exactly, the sum of the units above
    (plus the seed covariance's Cholesky check and the chi2 sum) applied to
    the track's own states: the counter counts nothing else.  (Whether an
    operation is trivial depends on values -- a landing remainder that rounds
    to 0, a direction with |T|^2 == 1, exact cancellations in the smoother's
    differences -- so two tracks with the same RKN trial counts may differ by
    a few percent; the decomposition holds track by track.)"""
    ev = synth.make_config(cfg, 12)
    for t in range(ev.n_tracks):
        st, units, total = oracle.count_units(ev, t)
        assert st == 0
        assert np.array_equal(units.sum(axis=0), total), (cfg, t)
        assert np.array_equal(total, oracle.count_ops(ev.subset(np.array([t])))[0])
        # the seed covariance is diagonal: its Cholesky check is six square roots
        assert units[0].tolist() == [0, 0, 0, 6, 0]
        n = int(ev.hit_offsets[t + 1] - ev.hit_offsets[t])
        assert units[5].tolist() == [n - 1, 0, 0, 0, 0]


def test_count_discs_close_to_planes():
    """The disc workload (C7, C2 measured in polar coordinates) costs per hit
    within 2 % to 10 % more than C2: the same fit plus the polar local frame
    (a sine/cosine into and an arctangent out of every transport) -- a guard
    against counting a different fit (e.g. discs taken for planes)."""
    e2 = synth.make_config(2, 200)
    e7 = synth.make_config(7, 200)
    c2 = oracle.count_ops(e2)[:, :4].sum(1) / np.diff(e2.hit_offsets)
    c7 = oracle.count_ops(e7)[:, :4].sum(1) / np.diff(e7.hit_offsets)
    r = c7.mean() / c2.mean()
    assert 1.02 < r < 1.10, r
