"""Pins of the oracle's storage-rounding emulation: binary16 rounding against
numpy's float16 conversion (round to nearest, ties to even) across normal,
subnormal, tie and overflow cases; the FP32 and scaled-FP16 deviation storage
against numpy casts; idempotence of a stored run."""
import numpy as np

S = np.array([1] + [3] * 4 + [5] * 4)


def test_round_f16_matches_numpy(orc):
    rng = np.random.default_rng(0)
    xs = list(rng.standard_normal(2000) * 10.0 ** rng.uniform(-9, 4, 2000))
    # exact midpoints between neighbouring binary16 values (ties to even)
    for m in (1.0, 0.75, 3.0e-5, 6.1e-5, 1.0e-7):
        h = np.float16(m)
        nxt = np.nextafter(h, np.float16(np.inf))
        xs.append((float(h) + float(nxt)) / 2)
        xs.append(-(float(h) + float(nxt)) / 2)
    xs += [65504.0, 65519.99, 65520.0, 1e9, -1e9, 2.0 ** -24, 2.0 ** -25, 2.0 ** -25 * 1.0000001, 0.0, -0.0]
    for x in xs:
        with np.errstate(over="ignore"):
            want = float(np.float64(x).astype(np.float16))
        got = orc.round_f16(x)
        assert got == want or (np.isinf(want) and np.isinf(got) and np.sign(got) == np.sign(want)), (x, got, want)


def test_round_storage_forms(orc):
    W = orc.weights()
    rng = np.random.default_rng(1)
    n = 8
    f = W[:, None, None] * (1 + 0.05 * rng.standard_normal((9, n, n)))
    p = orc.Params(n, n, 0.9)
    g = f - W[:, None, None]
    f32 = orc.round_storage(p, f, "f32")
    assert np.abs(f32 - (W[:, None, None] + g.astype(np.float32).astype(np.float64))).max() == 0.0
    f16 = orc.round_storage(p, f, "f16")
    want16 = W[:, None, None] + (g * 2.0 ** S[:, None, None]).astype(np.float16).astype(np.float64) / 2.0 ** S[:, None, None]
    assert np.abs(f16 - want16).max() == 0.0


def test_stored_run_is_representable(orc):
    from paper_1507_02509_amd import inputs
    n = 16
    ux, uy = inputs.spectral(n, 2, 0.05, seed=4)
    p = orc.Params(n, n, 0.95, collision=orc.KBC, variant=orc.KBC_B)
    for form in ("f32", "f16"):
        f = orc.run(p, orc.round_storage(p, orc.init(p, ux, uy), form), 5, storage=form)
        assert np.array_equal(orc.round_storage(p, f, form), f)
