"""The learned-proposal form over seeded exemplars (the 256^2 -> 512^2
workload's finest level): trained on pairs the plain method generates, the
learned forms (exact FP32 scan of the proposed leaves, BF16 scans with the
exact top-8, and the one-pass BF16 scan with class-minimum candidates; each
re-ranked in full dimension) stay within 1 % of exhaustive search at every
one of ten iterates from a held-out initial output, and below the plain
tree's gap; two of the sixteen exemplars."""
import pytest

pytestmark = pytest.mark.gpu


def test_learned_suite_two_exemplars(gpu_ctx):
    from paper_2006_11851_amd import learned_suite

    print("case: learned suite seeds 100, 101", flush=True)
    rows = learned_suite.run(gpu_ctx, [100, 101], log=lambda m: print(m, flush=True))
    for r in rows:
        assert r["pairs"] >= 120000
        for form in ("learned", "learned_bf16", "learned_bf16_class"):
            G = r[form]["gaps"]
            print(form, ["%.4f" % g for g in G], flush=True)
            assert max(G) <= 0.01, (form, G)
            assert r[form]["max_gap"] < r["tree"]["max_gap"]
