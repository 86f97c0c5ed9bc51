"""The allocation-free refinement, ebsd_refine_orientations_noalloc, against
ebsd_refine_orientations through the C ABI.  Both run the same kernels on
the same inputs, so their outputs must agree bit for bit (orientations,
peak heights and shifts), on two calls in a row where the second is smaller
and runs over the scratch the first one left; a batch beyond the static
scratch is rejected before anything is enqueued (outputs untouched)."""

import numpy as np
import pytest
import torch

from fixtures import configs, perturb_quats

from .gpu_util import banner, dev, host, tm

pytestmark = pytest.mark.gpu


def _inputs(n, p, seed):
    cfg = configs.tiny(p=p, l=8, n=n, seed=seed)
    q0 = perturb_quats(np.random.default_rng(seed), cfg["true_q"], 2.0)
    return cfg, q0


def _outputs(p):
    return dict(q=torch.full((p, 4), -7.0, dtype=torch.float64, device="cuda:0"),
                peak_h=torch.full((p,), -7.0, dtype=torch.float32, device="cuda:0"),
                shift=torch.full((p, 2), -7.0, dtype=torch.float32, device="cuda:0"))


@pytest.mark.parametrize("n", [64, 128, 160, 256])
def test_noalloc_refine_equals_refine_orientations(n):
    banner("refine noalloc n=%d" % n)
    t = tm()
    prm = t.params_default(max_shift=12 if n == 256 else -1)
    for call, p in enumerate((11, 4)):          # the second call is smaller
        cfg, q0 = _inputs(n, p, seed=40 + n + call)
        pats, master = dev(cfg["patterns"].float()), dev(cfg["master"])
        pcs, qi = dev(cfg["pcs"]), dev(q0)
        ref = t.refine_orientations(pats, master, cfg["pc"], qi, pc_per=pcs, prm=prm)
        got = t.refine_orientations(pats, master, cfg["pc"], qi, pc_per=pcs, prm=prm, out=_outputs(p),
                                    noalloc=True)
        torch.cuda.synchronize()
        for key in ("q", "peak_h", "shift"):
            assert torch.equal(got[key], ref[key]), (n, call, key)
        q = host(got["q"])
        assert np.allclose(np.linalg.norm(q, axis=1), 1.0, atol=1e-12) and np.all(np.isfinite(host(got["shift"])))
        print("[gpu]   n=%d call %d: P=%d bit-identical" % (n, call, p), flush=True)


def test_noalloc_rejects_batches_beyond_the_scratch():
    t = tm()
    import paper_1807_11313_amd as pkg
    n, p = 64, 5000                      # ~69 KB per pattern at 64 x 64: 5,000 exceed 256 MiB
    pats = torch.zeros((p, n, n), dtype=torch.float32, device="cuda:0")
    master = dev(configs.tiny(p=1, l=1).get("master"))
    q = torch.zeros((p, 4), dtype=torch.float64, device="cuda:0")
    q[:, 0] = 1.0
    out = _outputs(p)
    with pytest.raises(pkg.EbsdError) as e:
        t.refine_orientations(pats, master, (0.5, 0.5, 0.6), q, out=out, noalloc=True)
    assert e.value.code == -1 and "static" in str(e.value)
    torch.cuda.synchronize()
    assert torch.all(out["q"] == -7.0) and torch.all(out["peak_h"] == -7.0)
