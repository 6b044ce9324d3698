"""Pins of the low-precision emulation: bfloat16 rounding against its
definition on hand-picked values, the hi/lo split against exact identities,
and the emulated ladder term reducing to the FP64 one when the operands are
exactly representable."""
import numpy as np

import oracle as O
from oracle import precision_oracle as Pr
import ppl_synth as S


def test_bf16_rounding_hand_values():
    # bf16 keeps 8 significant bits: 1 + 2^-8 is a tie that rounds to even (1.0),
    # 1 + 3*2^-8 is a tie that rounds up to 1 + 2^-6; 1 + 2^-7 is representable
    vals = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -7, -3.0 - 2 ** -9, 0.0])
    want = np.array([1.0, 1.0, 1.0 + 2 ** -6, 1.0 + 2 ** -7, -3.0, 0.0])
    np.testing.assert_array_equal(Pr.round_bf16(vals), want)


def test_split_identities():
    x = np.random.default_rng(0).standard_normal(1000)
    hi, lo = Pr.split_bf16x3(x)
    x32 = Pr.round_fp32(x)
    assert np.array_equal(Pr.round_bf16(hi), hi) and np.array_equal(Pr.round_bf16(lo), lo)
    # hi + lo carries 16 significant bits: |x32 - hi - lo| <= 2^-16 |x32| (plus rounding of lo)
    assert np.all(np.abs(x32 - hi - lo) <= 2.0 ** -16 * np.abs(x32) + 1e-300)
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(hi) + 1e-300)


def test_split_bf16x6_identities():
    # an FP32 significand of 24 bits splits into three bf16 terms of 8 bits with no rest:
    # hi takes the leading 8 bits (rounded), leaving at most 16 bits, of which mid takes 8
    # and lo the remaining at most 8
    x = np.random.default_rng(2).standard_normal(1000) * np.exp(np.random.default_rng(3).uniform(-20, 20, 1000))
    hi, mid, lo = Pr.split_bf16x6(x)
    x32 = Pr.round_fp32(x)
    for part in (hi, mid, lo):
        assert np.array_equal(Pr.round_bf16(part), part)
    np.testing.assert_array_equal(hi + mid + lo, x32)
    assert np.all(np.abs(mid) <= 2.0 ** -8 * np.abs(hi) + 1e-300)
    assert np.all(np.abs(lo) <= 2.0 ** -8 * np.abs(mid) + 1e-300)
    # hi and mid are the two terms of the bf16x3 split
    h3, l3 = Pr.split_bf16x3(x)
    assert np.array_equal(h3, hi) and np.array_equal(l3, mid)
    # the six kept products carry x*y to about 2^-24 relative: the dropped mid*lo and lo*mid
    # are each at most 2^-24 |hi*hi|, lo*lo at most 2^-32 |hi*hi|
    y = np.random.default_rng(4).standard_normal(1000)
    a, b = Pr.split_bf16x6(x), Pr.split_bf16x6(y)
    six = a[0] * b[0] + a[0] * b[1] + a[1] * b[0] + a[1] * b[1] + a[0] * b[2] + a[2] * b[0]
    exact = x32 * Pr.round_fp32(y)
    assert np.all(np.abs(six - exact) <= 3 * 2.0 ** -24 * np.abs(exact) + 1e-300)


def test_emulation_is_exact_on_representable_inputs():
    # small integers are exact in bf16: every rounding point is then exact
    o, v = 2, 5
    rng = np.random.default_rng(1)
    L = rng.integers(-3, 4, size=(3, o + v, o + v)).astype(float)
    L = L + L.transpose(0, 2, 1)
    t = rng.integers(-2, 3, size=(o, o, v, v)).astype(float)
    t = t + t.transpose(1, 0, 3, 2)
    R = O.ppl(L, o, t)
    for prec in ("fp32", "bf16x3", "bf16x6"):
        np.testing.assert_array_equal(Pr.ppl_lowprec(L, o, t, prec), R)


def test_emulated_error_levels():
    s = S.make_system(4, 16, 48, 2)
    t = O.mp2_amplitudes(s["L"], 4, s["e_occ"], s["e_vir"])
    R = O.ppl(s["L"], 4, t)
    e32 = np.linalg.norm(Pr.ppl_lowprec(s["L"], 4, t, "fp32") - R) / np.linalg.norm(R)
    eb = np.linalg.norm(Pr.ppl_lowprec(s["L"], 4, t, "bf16x3") - R) / np.linalg.norm(R)
    e6 = np.linalg.norm(Pr.ppl_lowprec(s["L"], 4, t, "bf16x6") - R) / np.linalg.norm(R)
    assert 1e-9 < e32 < 1e-6
    assert e32 < eb < 1e-4
    # bf16x6 drops only products below 2^-24 of the leading one: it stays at the FP32 level
    # (its rounding points are those of FP32), where dropping any kept product (say mid*mid,
    # 2^-16) would put it near the bf16x3 level
    assert 0.5 * e32 < e6 < 2.0 * e32
    assert e6 < eb / 10


def test_planted_dropped_product_fails_the_level_pin(monkeypatch):
    """A bf16x6 emulation that dropped one kept product (mid*mid) would leave the FP32
    level that the error-level pin requires."""
    s = S.make_system(4, 16, 48, 2)
    t = O.mp2_amplitudes(s["L"], 4, s["e_occ"], s["e_vir"])
    R = O.ppl(s["L"], 4, t)
    e32 = np.linalg.norm(Pr.ppl_lowprec(s["L"], 4, t, "fp32") - R) / np.linalg.norm(R)
    good = Pr._mul_form

    def planted(prec):
        prep, mm = good(prec)
        if prec == "bf16x6":
            def mm(a, b):
                return a[0] @ b[0].T + a[0] @ b[1].T + a[1] @ b[0].T + a[0] @ b[2].T + a[2] @ b[0].T
        return prep, mm

    monkeypatch.setattr(Pr, "_mul_form", planted)
    e6 = np.linalg.norm(Pr.ppl_lowprec(s["L"], 4, t, "bf16x6") - R) / np.linalg.norm(R)
    assert not e6 < 2.0 * e32
