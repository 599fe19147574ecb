"""The polynomial tables of the device math (csrc/pes_poly.hpp) against the
functions they stand for, evaluated on the host in FP64 by the same Horner
scheme as the kernels, with an mpmath reference at 30 digits."""
import math
import os
import re

import mpmath as mp
import numpy as np
import pytest

POLY = os.path.join(os.path.dirname(__file__), "..", "paper_2602_12011_amd", "csrc", "pes_poly.hpp")


def _tables():
    text = open(POLY).read()
    arrays = {m.group(1): [float(x) for x in m.group(3).replace("\n", " ").split(",") if x.strip()]
              for m in re.finditer(r"constexpr double (\w+)\[(\d+)\] = \{([^}]*)\}", text)}
    arrays.update({m.group(1): [float(x.strip().rstrip("f")) for x in m.group(3).replace("\n", " ").split(",")
                                if x.strip()]
                   for m in re.finditer(r"constexpr float (\w+)\[(\d+)\] = \{([^}]*)\}", text)})
    scalars = {m.group(1): float(m.group(2))
               for m in re.finditer(r"constexpr double (\w+) = ([-+0-9.eE]+);", text)}
    return arrays, scalars


def _horner(c, t):
    acc = np.full_like(t, c[0])
    for k in c[1:]:
        acc = acc * t + k
    return acc


mp.mp.dps = 30
ARR, SCAL = _tables()
X_SMALL0 = SCAL["kClassBMax0"] / (2.0 * math.sqrt(3.0))

# (table, function of the variable, variable range, t = variable^2)
CASES = [
    ("kSin2pi", lambda y: mp.sin(2 * mp.pi * y) / y, 0.125),
    ("kCos2pi", lambda y: mp.cos(2 * mp.pi * y), 0.125),
    ("kSincShort", lambda b: mp.sin(b) / b, math.sqrt(SCAL["kSincShortTMax"])),
    ("kSincLong", lambda b: mp.sin(b) / b, math.sqrt(SCAL["kSincLongTMax"])),
    ("kSinSmall", lambda x: mp.sin(x) / x, math.sqrt(SCAL["kSmallTMax"])),
    ("kCosSmall", lambda x: mp.cos(x), math.sqrt(SCAL["kSmallTMax"])),
    ("kSincC0", lambda b: mp.sin(b) / b, SCAL["kClassBMax0"]),
    ("kSinSmallC0", lambda x: mp.sin(x) / x, X_SMALL0),
    ("kCosSmallC0", lambda x: mp.cos(x), X_SMALL0),
]


@pytest.mark.parametrize("name,fn,vmax", CASES, ids=[c[0] for c in CASES])
def test_fit_accuracy(name, fn, vmax):
    v = np.linspace(vmax * 1e-6, vmax, 2001)
    got = _horner(ARR[name], v * v)
    ref = np.array([float(fn(mp.mpf(float(x)))) for x in v])
    scale = np.max(np.abs(ref))
    err = np.max(np.abs(got - ref)) / scale
    # fit error (<= 3e-16) plus the rounding of the FP64 Horner evaluation
    assert err < 1e-15, (name, err)


def test_short_range_class_is_narrower():
    # the short-range fits must cover every argument a class-0 wavefront produces:
    # link sinc a (1 -+ k.n) <= 2 pi f L, arm phase |pi f k.Delta| <= pi f L / sqrt 3
    assert SCAL["kClassBMax0"] ** 2 <= SCAL["kSincShortTMax"]
    assert X_SMALL0 ** 2 <= SCAL["kSmallTMax"]
    assert len(ARR["kSincC0"]) < len(ARR["kSincShort"])
    assert len(ARR["kSinSmallC0"]) < len(ARR["kSinSmall"])


# FP32 tables of the single-precision kernels: evaluated by the same Horner
# scheme in float32 (coefficients rounded to float32 as the device holds them)
CASES_F32 = [
    ("kSin2piF", lambda y: mp.sin(2 * mp.pi * y) / y, 0.125),
    ("kCos2piF", lambda y: mp.cos(2 * mp.pi * y), 0.125),
    ("kSincShortF", lambda b: mp.sin(b) / b, math.sqrt(SCAL["kSincShortTMax"])),
    ("kSincLongF", lambda b: mp.sin(b) / b, math.sqrt(SCAL["kSincLongTMax"])),
    ("kSinSmallF", lambda x: mp.sin(x) / x, math.sqrt(SCAL["kSmallTMax"])),
    ("kCosSmallF", lambda x: mp.cos(x), math.sqrt(SCAL["kSmallTMax"])),
    ("kSincC0F", lambda b: mp.sin(b) / b, SCAL["kClassBMax0"]),
    ("kSinSmallC0F", lambda x: mp.sin(x) / x, X_SMALL0),
    ("kCosSmallC0F", lambda x: mp.cos(x), X_SMALL0),
]


@pytest.mark.parametrize("name,fn,vmax", CASES_F32, ids=[c[0] for c in CASES_F32])
def test_fit_accuracy_f32(name, fn, vmax):
    v = np.linspace(vmax * 1e-6, vmax, 2001).astype(np.float32)
    c = np.asarray(ARR[name], dtype=np.float32)
    t = v * v
    acc = np.full_like(t, c[0])
    for k in c[1:]:
        acc = (acc * t + k).astype(np.float32)
    ref = np.array([float(fn(mp.mpf(float(x)))) for x in v])
    err = np.max(np.abs(acc.astype(np.float64) - ref)) / np.max(np.abs(ref))
    # fit error (<= 3e-8) plus the rounding of a float32 Horner evaluation
    assert err < 4e-7, (name, err)
    assert len(ARR[name]) < len(ARR[name[:-1]])    # fewer terms than the FP64 fit of the same function
