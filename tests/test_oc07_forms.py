"""The turbulent term of eq:dv as the kernel writes it (gd_physics.hpp,
oc07_dv2_r), its steps evaluated on the host, against the closed forms of
Ormel & Cuzzi (2007) for St1 >= St2 (Sect. 2.5.2) evaluated exactly in
rational arithmetic:

* tight (St1 < t = Re^-1/2): Vg^2 (St1 - St2)/(St1 + St2) (St1^2/(St1 + t) -
  St2^2/(St2 + t)), the kernel's form being the same quotient rearranged over
  (St1 + St2)(St1 + t)(St2 + t);
* intermediate (t <= St1 < 1, y_a = 1.6): Vg^2 St1 [2 y_a - (1 + e) +
  2/(1 + e) (1/(1 + y_a) + e^3/(y_a + e))] with e = St2/St1, the kernel's
  form that expression multiplied through by St1^3 into one quotient;
* heavy (St1 >= 1): Vg^2 (1/(1 + St1) + 1/(1 + St2)).

The kernel's quotients come from the hardware reciprocal with Newton steps,
within 1 ulp of the rounded quotient taken here; the bound below (8 ulp)
covers that and the few roundings of each form.  A form with a dropped term,
a wrong sign or swapped St fails by many orders more."""
import math
import random
from fractions import Fraction as Fr

YA = 1.6


def _kernel(St1, St2, Vg2, tke):
    """The kernel's steps in its order (tight and intermediate one quotient
    each), with correctly rounded quotients."""
    dSt = St1 - St2
    if St1 < tke:
        num = St1 * St2 + tke * (St1 + St2)
        den = (St1 + St2) * (St1 + tke) * (St2 + tke)
        return (Vg2 * (dSt * dSt) * num) / den
    if St1 < 1.0:
        u = YA * St1 + St2
        num = 2.0 * (St1 * St1 * u * (1.0 / (1.0 + YA)) + St2 * St2 * St2)
        return Vg2 * (((2.0 * YA - 1.0) * St1 - St2) + num / ((St1 + St2) * u))
    return Vg2 * (1.0 / (1.0 + St1) + 1.0 / (1.0 + St2))


def _published(St1, St2, Vg2, tke):
    """The closed forms as published, in exact arithmetic on the same float
    inputs (y_a taken as the double nearest 1.6, as the kernel has it)."""
    a, b, V, t, ya = Fr(St1), Fr(St2), Fr(Vg2), Fr(tke), Fr(YA)
    if St1 < tke:
        return V * (a - b) / (a + b) * (a * a / (a + t) - b * b / (b + t))
    if St1 < 1.0:
        e = b / a
        br = 2 * ya - (1 + e) + 2 / (1 + e) * (1 / (1 + ya) + e ** 3 / (ya + e))
        return V * br * a
    return V * (1 / (1 + a) + 1 / (1 + b))


def _cases(seed, n):
    rng = random.Random(seed)
    for _ in range(n):
        tke = 10 ** rng.uniform(-4, -1)
        regime = rng.randrange(3)
        if regime == 0:
            St1 = tke * rng.uniform(1e-3, 0.999)
        elif regime == 1:
            St1 = rng.uniform(tke, 0.999)
        else:
            St1 = 10 ** rng.uniform(0, 3)
        # close pairs (the drift-free limit) and distant ones
        St2 = St1 * (1 - 10 ** rng.uniform(-12, -1)) if rng.random() < 0.5 else St1 * rng.random() ** 3
        yield St1, St2, 10 ** rng.uniform(2, 10), tke


def test_kernel_forms_match_published_in_every_regime():
    seen = [0, 0, 0]
    worst = 0.0
    for St1, St2, Vg2, tke in _cases(7, 3000):
        seen[0 if St1 < tke else (1 if St1 < 1.0 else 2)] += 1
        want = float(_published(St1, St2, Vg2, tke))
        got = _kernel(St1, St2, Vg2, tke)
        if want == 0.0:
            assert got == 0.0
            continue
        worst = max(worst, abs(got - want) / math.ulp(want))
    assert min(seen) > 500, seen
    assert worst <= 8.0, worst


def test_equal_grains():
    """Equal Stokes numbers: zero in the tight regime (no relative motion),
    Vg^2 St (2 y_a - 2 + 2 (1/(1 + y_a) + 1/(y_a + 1))/2) = Vg^2 St (2 y_a - 2 +
    2/(1 + y_a)) in the intermediate one, 2 Vg^2/(1 + St) in the heavy one."""
    tke = 1e-2
    assert _kernel(5e-3, 5e-3, 3.0, tke) == 0.0
    St = 0.3
    want = 3.0 * St * (2 * YA - 2 + 2 / (1 + YA))
    assert abs(_kernel(St, St, 3.0, tke) - want) <= 4 * math.ulp(want)
    assert abs(_kernel(4.0, 4.0, 3.0, tke) - 6.0 / 5.0) <= 2 * math.ulp(1.2)
