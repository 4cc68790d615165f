"""The seeded input recipes: the batched-boxes and local-box workloads are
deterministic and follow their stated distributions."""
import math

import numpy as np

import workloads


def test_box_batch_recipe():
    a = workloads.box_batch(3, nbox=64)
    b = workloads.box_batch(3, nbox=64)
    assert len(a) == 64
    ns = np.array([len(s["x"]) for _, s, _ in a])
    assert ns.min() >= 2 ** 10 - 1 and ns.max() <= 2 ** 16 + 1
    for (pa, sa, da), (pb, sb, db) in zip(a, b):
        assert da == db and pa["alpha"] == pb["alpha"] and np.array_equal(sa["x"], sb["x"])
        assert 1e-4 <= pa["alpha"] <= 1e-2 and 100.0 <= pa["v_frag"] <= 1000.0
        R, side = pa["R_box"], pa["L"][0]
        assert 10 * workloads.AU <= R <= 100 * workloads.AU and math.isclose(side, 0.005 * R)
        assert pa["periodic"] == (1, 1, 1) and pa["push"] == "none" and pa["kernel"] == "physical"
        # positions inside the periodic cube, grain radii 1 um .. 1 mm
        assert sa["x"].min() >= R and sa["x"].max() < R + side
        assert np.abs(sa["y"]).max() <= side / 2 and np.abs(sa["z"]).max() <= side / 2
        radius = 0.5 * np.cbrt(6.0 * sa["m"] / (math.pi * pa["rho_s"]))
        assert radius.min() >= 1e-4 * (1 - 1e-9) and radius.max() <= 1e-1 * (1 + 1e-9)
    # log-uniform sizes: the median of log2 N sits near 13
    assert abs(np.median(np.log2(ns)) - 13.0) < 1.0


def test_local_box_dust_mass():
    p = workloads.local_box_params(2048, R_au=30.0)
    s = workloads.local_box(1, 2048, p)
    R = 30.0 * workloads.AU
    sigma = p["Sigma_g0"] * (R / p["R0"]) ** p["p"]
    rho_g = sigma / (math.sqrt(2.0 * math.pi) * p["h_g0"] * R)
    assert math.isclose(s["M"].sum(), 0.01 * rho_g * p["L"][0] ** 3, rel_tol=1e-12)


def test_diffusion_ring_recipe():
    # the dust ring of Sect. 3.2: ln(R/R0) ~ N(0, 0.05^2), midplane, at rest
    import math

    import numpy as np

    st = workloads.diffusion_ring(3, 1 << 16)
    lnR = np.log(st["r"])
    assert abs(lnR.mean()) < 5 * 0.05 / 256 and abs(lnR.std() - 0.05) < 5 * 0.05 / math.sqrt(2 * (1 << 16))
    assert np.all(st["th"] == 0.5 * math.pi) and not st["vr"].any() and not st["lph"].any()
    assert len(np.unique(st["id"])) == len(st["id"])
    np.testing.assert_allclose(np.hypot(st["x"], st["y"]), st["r"], rtol=1e-15)
    p = workloads.diffusion_ring_params("density", St=10.0)
    assert (p["h_g0"], p["p"], p["q"], p["alpha"], p["St_diff"], p["vint"]) == (0.05, -1.0, 0.5, 0.04, 10.0, 1)
    # nu = alpha h_g0^2 sqrt(GM R0) (R/R0)^2 = 1e-4 (R/R0)^2 in code units
    assert abs(p["alpha"] * p["h_g0"] ** 2 * math.sqrt(p["GM"] * p["R0"]) - 1e-4) < 1e-18
