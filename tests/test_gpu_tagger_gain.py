"""What the trained tagger gains over the plain criterion (a project
addition): trained on the GPU by the library's own kernels on labels from
plain-tagger runs, it regrids half as often as plain tagging every 4 coarse
steps and still ends with a smaller pressure error against the exact
solution than plain tagging at the same (8-step) interval and than the
4-step plain run."""
import os

import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    torch = pytest.importorskip("torch")
    if not os.path.exists("/dev/kfd"):
        pytest.skip("no GPU on this machine")
    assert torch.cuda.is_available(), "GPU present but torch.cuda.is_available() is False"


def test_learned_tagger_gain():
    import paper_2205_07572_amd as af
    from paper_2205_07572_amd import tagger_train as tt
    from paper_2205_07572_amd.amr import TagRule
    wl = tt.Workload(rule=TagRule(af.TAG_GRADIENT, 0, 3.0, 1.0))
    x, y = tt.generate(wl, range(4), horizon=8)
    tagger, losses = tt.train(x, y, steps=600)
    assert losses[-1] < 0.5 * losses[0]
    xv, yv = tt.generate(wl, range(200, 201), horizon=8)
    acc, conf = tt.accuracy(tagger, xv, yv)
    ev = tt.evaluate(wl, range(200, 202), tagger, horizon=8)
    print(f"[tagger-gain] held-out accuracy {acc:.3f}; {ev}", flush=True)
    p4, l8, p8 = ev["plain_every4"], ev["learned_every8"], ev["plain_every8"]
    assert acc > 0.8
    assert conf[2][2] >= 0.9 * sum(conf[2])  # refine recall
    assert l8["regrids"] <= 0.5 * p4["regrids"] + 1
    assert l8["linf_p"] < 0.7 * p8["linf_p"]
    assert l8["linf_p"] < p4["linf_p"]
