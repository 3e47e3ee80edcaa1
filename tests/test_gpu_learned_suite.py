"""The learned-proposal form over seeded exemplars (the 256^2 -> 512^2
workload's finest level): trained on pairs the plain method generates, its
energy gap to exhaustive search stays below the plain tree's; with BF16
scans and the full-dimension re-rank it is within 1.5 % at the initial
output and within 1 % from the third iteration on; two of the sixteen
exemplars."""
import pytest

pytestmark = pytest.mark.gpu


def test_learned_suite_two_exemplars(gpu_ctx):
    from paper_2006_11851_amd import learned_suite

    print("case: learned suite seeds 100, 101", flush=True)
    rows = learned_suite.run(gpu_ctx, [100, 101], log=lambda m: print(m, flush=True))
    for r in rows:
        assert r["pairs"] >= 120000
        assert r["learned"]["max_gap"] < r["tree"]["max_gap"]
        assert r["learned_bf16"]["max_gap"] < r["tree"]["max_gap"]
        G = r["learned_bf16"]["gaps"]
        assert G[0] <= 0.015 and max(G[2:]) <= 0.01, G
