"""The allocation-free entry point (pc_hac_noalloc) against pc_hac: the same
rows (average linkage: heights within 1e-12 relative, the bar for any cache
size), on two calls in a row whose second input is smaller, for every
linkage and for the grid, box-tree and Gram searches. The scratch array keeps
the first call's contents, so the second call also shows that everything it
needs starts cleared."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    assert torch.cuda.is_available()
    import paper_2106_04727_amd as pc
    from paper_2106_04727_amd import parchain

    pc.load_library()
    return pc, parchain, torch


def same_rows(Za, Zb, link):
    if link != "average":
        return np.array_equal(Za, Zb)
    return (np.array_equal(Za[:, [0, 1, 3]], Zb[:, [0, 1, 3]])
            and np.allclose(Za[:, 2], Zb[:, 2], rtol=1e-12, atol=0.0))


def run_noalloc(parchain, torch, ctx, x, link, **kw):
    dev = torch.device("cuda:0")
    xt = torch.from_numpy(np.ascontiguousarray(x, np.float32)).to(dev)
    n, d = x.shape
    rows = torch.empty((max(n - 1, 1), 4), dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev).cuda_stream
    torch.cuda.synchronize()
    st = ctx.hac_noalloc(xt.data_ptr(), n, d, link, rows.data_ptr(), stream=stream, **kw)
    torch.cuda.synchronize()
    return parchain.rows_to_Z(rows[: n - 1]), st


@pytest.mark.parametrize("link,d,n1,n2,kind", [
    ("ward", 2, 60_000, 9_000, "b"),
    ("avgsq", 2, 40_000, 7_000, "b"),
    ("complete", 2, 30_000, 5_000, "b"),
    ("average", 2, 12_000, 3_000, "b"),
    ("ward", 5, 20_000, 4_000, "u"),      # box tree, then Gram search
    ("complete", 10, 8_000, 2_000, "b"),  # Gram search, interval tiles
    ("average", 64, 4_000, 1_500, "s"),   # Gram search at d = 64
])
def test_noalloc_equals_pc_hac(env, link, d, n1, n2, kind):
    pc, parchain, torch = env
    ctx = parchain.Context(0)
    for i, n in enumerate((n1, n2)):
        seed = 300 + 7 * i + d
        if kind == "b":
            x = synth.blobs(n, d, 30, 0.02, seed)
        elif kind == "u":
            x = synth.uniform(n, d, seed)
        else:
            x = synth.sphere_blobs(n, d, 20, 0.1, seed)
        print("noalloc %s d=%d n=%d call %d" % (link, d, n, i + 1), flush=True)
        Zn, st = run_noalloc(parchain, torch, ctx, x, link)
        Zr = pc.hac(x, link)
        assert Zn.shape == (n - 1, 4)
        assert same_rows(Zn, Zr, link), (link, d, n, i)
    ctx.close()


def test_noalloc_rejects_inputs_beyond_the_scratch(env):
    pc, parchain, torch = env
    from paper_2106_04727_amd import PCError

    ctx = parchain.Context(0)
    x = synth.uniform(3_000_000, 2, 5)
    with pytest.raises(PCError) as e:
        run_noalloc(parchain, torch, ctx, x, "complete")
    assert e.value.status == -3
    # the context still works afterwards, allocation-free and not
    x = synth.blobs(5_000, 2, 10, 0.02, 6)
    Zn, _ = run_noalloc(parchain, torch, ctx, x, "ward")
    assert np.array_equal(Zn, pc.hac(x, "ward"))
    ctx.close()
