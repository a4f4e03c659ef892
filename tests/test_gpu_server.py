"""Serving on the GPU: requests of uneven n, d and linkage run concurrently
on several slots (own context and stream each); every result must equal the
same request clustered alone (pc_hac on an idle device), bit for bit."""
import numpy as np
import pytest

import oracle
import synth
from tests import _trees

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pc():
    import torch

    assert torch.cuda.is_available()
    import paper_2106_04727_amd as pc

    pc.load_library()
    return pc


def requests(seed=5):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(14):
        n = int(np.exp(rng.uniform(np.log(256), np.log(6000))))
        d = int(rng.choice([2, 3, 10, 64]))
        link = ["complete", "average", "ward", "avgsq"][i % 4]
        k = int(rng.integers(5, 101))
        sigma = float(rng.uniform(0.01, 0.05))
        out.append((synth.blobs(n, d, k, sigma, 100 + i), link))
    return out


def test_alone_equals_in_the_mix(pc):
    reqs = requests()
    alone = [pc.hac(x, link) for x, link in reqs]
    with pc.Server(device=0, slots=4) as srv:
        tickets = [srv.submit(x, link) for x, link in reqs]
        mixed = [srv.result(t)[0] for t in tickets]
        st = srv.stats()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert st["peak_running"] >= 2  # requests did share the device
    for (x, link), a, m in zip(reqs, alone, mixed):
        assert np.array_equal(a, m), (x.shape, link)
    # and two of them against the oracle
    for (x, link), m in list(zip(reqs, mixed))[:2]:
        Zo, _ = oracle.nnchain(x, link, threads=8)
        assert _trees.same_tree(m, Zo, x.shape[0], rtol={"average": 1e-12, "avgsq": 1e-10}.get(link, 0.0))


def test_failed_request_does_not_stop_the_server(pc):
    from paper_2106_04727_amd import PCError

    x = synth.uniform(500, 3, 1)
    bad = x.copy()
    bad[7, 1] = np.nan
    with pc.Server(device=0, slots=2) as srv:
        tb = srv.submit(bad, "ward")
        tg = srv.submit(x, "ward")
        with pytest.raises(PCError) as e:
            srv.result(tb)
        assert e.value.status == -2
        Z, _ = srv.result(tg)
    assert np.array_equal(Z, pc.hac(x, "ward"))
