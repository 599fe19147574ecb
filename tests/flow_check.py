"""Row-by-row check of one pass of the coupling flow, as the library computed
it (pes_flow_probe: the FP32 state at every layer boundary and every layer's
conditioner stages), against the flow reference in oracle/flow.py.

The library's network products take BF16 operands and accumulate in FP32, in
an order of its own.  Each rounding to BF16 (of a conditioner input or a
hidden activation) is therefore only fixed up to the accumulation error: where
the exact value lies within that error of a rounding midpoint, either
neighbour is a correct result, and a different choice moves the pass's output
by up to ~1e-2.  So every stage is checked on the values the library itself
fed it, against the exact interval the reference admits:

  start   slot 0 equals the reference's standardized rows (forward) or the
          FP32 latent (inverse);
  a0      the BF16 conditioner input is exactly the rounding of the state's
          conditioning coordinates;
  a1, a2  each hidden BF16 value lies in [bf16(relu(v - e)), bf16(relu(v + e))]
          with v = a W + b in FP64 and e = (K + 2) 2^-24 (|a| |W| + |b|), the
          bound of an FP32 accumulation of K products in any order;
  o       |o - v| <= e;
  layer   the transformed coordinates agree with the reference coupling of
          that o to 4e-6 (|x e^s| + |t|) (FP32 tanh, exp, fma), the others are
          unchanged, and the running log det grows by the reference's sum s;
  end     z and log q (forward) or theta and log det (inverse) follow from the
          last slot.

Then the pass end to end against the reference's own chain from its own
inputs: every row whose rounding decisions all equal the reference's agrees to
5e-5 (out) and 1e-4 (log q) (FP32 state arithmetic through eight layers; an
FP32 emulation stays within 7e-6 over 3000 rows); a row where some decision
went the other way at an admissible near-tie is held by the stage checks
above, row by row, and is only counted.  No row is exempt from a check.
"""
import numpy as np

U32 = 2.0 ** -24
N_ACT = 576
A0, A1, A2, AO = slice(0, 32), slice(32, 288), slice(288, 544), slice(544, 576)


def _interval_ok(F, got, v, e):
    lo = F.bf16(np.maximum(v - e, 0.0))
    hi = F.bf16(np.maximum(v + e, 0.0))
    return (got >= lo) & (got <= hi)


def check_pass(F, flat, inverse, x0, out, lq, st, ld, acts, mu=None, L=None, tau=1.0, what=""):
    """x0: the reference's own starting rows (standardized theta, or the FP32
    latent tau z); out, lq, st, ld, acts: the probe's results as numpy arrays.
    Returns (number of rows whose decisions differ from the reference chain,
    worst end-to-end error of the others).  Raises AssertionError on a
    mismatch."""
    st = np.asarray(st, dtype=np.float64)
    ld = np.asarray(ld, dtype=np.float64)
    acts = np.asarray(acts, dtype=np.float64)
    n = st.shape[1]
    assert st.shape == (9, n, 11) and ld.shape == (9, n) and acts.shape == (8, n, N_ACT)
    x0 = np.asarray(x0, dtype=np.float64)
    # start
    if inverse:
        assert np.array_equal(st[0], x0), (what, "latent")
        assert np.all(ld[0] == 0.0)
    else:
        assert np.all(np.abs(st[0] - x0) <= 2.0 ** -23 * np.abs(x0)), (what, "standardized rows")
        assert np.all(ld[0] == 0.0)
    for k, l in enumerate(F.layer_order(inverse)):
        C, T = F.cond_set(l), F.trans_set(l)
        nc, nt = len(C), len(T)
        x = st[k]
        a = acts[l]
        tag = (what, "layer", l)
        assert np.array_equal(a[:, A0][:, :nc], F.bf16(x[:, C])), tag + ("a0",)
        assert np.all(a[:, A0][:, nc:] == 0.0), tag + ("a0 padding",)
        v, sc = F.dense(flat, l, 1, a[:, A0][:, :nc])
        ok = _interval_ok(F, a[:, A1], v, (32 + 2) * U32 * sc)
        assert ok.all(), tag + ("a1", int((~ok).sum()))
        v, sc = F.dense(flat, l, 2, a[:, A1])
        ok = _interval_ok(F, a[:, A2], v, (256 + 2) * U32 * sc)
        assert ok.all(), tag + ("a2", int((~ok).sum()))
        v, sc = F.dense(flat, l, 3, a[:, A2])
        o = a[:, AO][:, :2 * nt]
        err = np.abs(o - v) / ((256 + 2) * U32 * sc + 1e-300)
        assert np.all(err <= 1.0), tag + ("o", float(err.max()))
        assert np.all(a[:, AO][:, 2 * nt:] == 0.0), tag + ("o padding",)
        y, ssum = F.coupling(l, x, o, inverse)
        s = 3.0 * np.tanh(o[:, :nt] / 3.0)
        t = o[:, nt:2 * nt]
        scale = (np.abs(x[:, T] * np.exp(s)) + np.abs(t)) if not inverse else \
            (np.abs(x[:, T]) + np.abs(t)) * np.exp(-s)
        err = np.abs(st[k + 1][:, T] - y[:, T]) / (4e-6 * scale + 1e-30)
        assert np.all(err <= 1.0), tag + ("coupling", float(err.max()))
        assert np.array_equal(st[k + 1][:, C], x[:, C]), tag + ("conditioning coordinates changed",)
        err = np.abs(ld[k + 1] - (ld[k] + ssum)) / (1e-6 * (np.abs(ld[k]) + np.abs(s).sum(axis=1)) + 1e-30)
        assert np.all(err <= 1.0), tag + ("log det", float(err.max()))
    # end
    if inverse:
        th = F.unstandardize(st[8], mu, L)
        assert np.all(np.abs(out - th) <= 1e-13 * np.maximum(1.0, np.abs(th))), (what, "theta")
        if lq is not None:
            assert np.array_equal(np.asarray(lq), ld[8]), (what, "log det out")
    else:
        assert np.array_equal(out, st[8]), (what, "z")
        ref = F.log_base(st[8], ld[8], tau) - np.log(np.diag(F.whitening(L))).sum()
        assert np.all(np.abs(lq - ref) <= 1e-12 * np.maximum(1.0, np.abs(ref))), (what, "log q")
    # end to end against the reference's own chain
    S, LD, R = F.trace(flat, x0, inverse)
    same = np.ones(n, dtype=bool)
    for l in range(F.N_LAYERS):
        nc = len(F.cond_set(l))
        same &= np.all(acts[l][:, A0][:, :nc] == R[l]["a0"], axis=1)
        same &= np.all(acts[l][:, A1] == R[l]["a1"], axis=1)
        same &= np.all(acts[l][:, A2] == R[l]["a2"], axis=1)
    e_out = (np.abs(st[8] - S[8]) / np.maximum(1.0, np.abs(S[8]))).max(axis=1)
    e_ld = np.abs(ld[8] - LD[8]) / np.maximum(1.0, np.abs(LD[8]))
    worst = float(max(e_out[same].max(initial=0.0), e_ld[same].max(initial=0.0)))
    bad = same & ((e_out > 5e-5) | (e_ld > 1e-4))
    assert not bad.any(), (what, "end to end", np.nonzero(bad)[0][:10], worst)
    return int((~same).sum()), worst
