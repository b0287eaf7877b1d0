"""The time march that trains and evaluates the learned initial guess, on a
small shell (N = Nr = 16, two-level RAS): every solve reaches ||r|| <= 1e-8
||b|| whatever its guess, Step 3 leaves a face divergence within that
tolerance, training lowers the loss, and the guesses are ranked by their
error against the solution."""
import pytest

pytestmark = pytest.mark.gpu


def test_march_small():
    from paper_2009_02171_amd import march
    r = march.run(n=16, nr=16, sub=(8, 8, 8), levels=2, train_steps=30, eval_steps=4, train_iters=8,
                  log=lambda m: print(m, flush=True))
    print(r)
    for name, s in r["systems"].items():
        for v in ("plain_a", "mixed_a", "mixed_b", "mixed_c"):
            assert s[v]["solves"] == 4
            assert s[v]["relres_max"] <= 1.0001e-8
        assert s["face_div_rel_max"] <= 1.0001e-8
        assert s["loss_last"] < 0.5 * s["loss_first"]
        q = s["guess_quality_median"]
        # extrapolation beats the previous solution; the trained network's own
        # guess has a smaller error than extrapolation
        assert q["err_extrap"] < 0.5 * q["err_prev"]
        assert q["err_net"] < q["err_extrap"]
        # with the fallback the learned form never starts from a larger residual
        assert s["mixed_c"]["res0_rel_median"] <= s["mixed_b"]["res0_rel_median"] * (1 + 1e-12)
