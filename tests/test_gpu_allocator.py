"""pg_set_allocator through the C ABI: torch's caching allocator serves every
device block of a build and a search (the device memory torch reports grows
while the tree lives), the results equal those made with the library's own
pool, and the allocator can be switched back once the tree is freed.  The
default allocator's block cache: results do not depend on its limit (a child
process with a 4 MiB limit trims at nearly every free) or on
pg_release_cached between calls."""
import gc

import numpy as np
import pytest

from paper_2207_01834_amd import datagen
from parity import say

pytestmark = pytest.mark.gpu


def test_torch_caching_allocator(dev):
    import torch

    import paper_2207_01834_amd._binding as pg
    gc.collect()
    pts = datagen.uniform_int(200_000, 3, seed=8)
    x = torch.from_numpy(pts).to(dev)
    t = pg.kdtree_build(x, leaf=16)
    ref_i, ref_d = t.knn_all(10)
    torch.cuda.synchronize()
    ref_i, ref_d = ref_i.cpu(), ref_d.cpu()
    del t
    gc.collect()
    say("switching to torch's caching allocator")
    pg.use_torch_allocator(True)
    try:
        before = torch.cuda.memory_allocated(dev)
        t = pg.kdtree_build(x, leaf=16)
        torch.cuda.synchronize()
        held = torch.cuda.memory_allocated(dev) - before
        assert held > 200_000 * 3 * 4  # the tree's arrays came from torch
        gi, gd = t.knn_all(10)
        torch.cuda.synchronize()
        assert torch.equal(gi.cpu(), ref_i) and torch.equal(gd.cpu(), ref_d)
        with pytest.raises(pg.PargeoError):
            pg.use_torch_allocator(False)  # the tree still holds blocks
        del t, gi, gd
        gc.collect()
        torch.cuda.synchronize()
    finally:
        pg.use_torch_allocator(False)
    assert torch.cuda.memory_allocated(dev) <= before + 16 * 1024 * 1024


def test_torch_allocator_bdl_sequence(dev):
    """A BDL-tree insert / erase / k-NN sequence (many staging and per-tree
    blocks, rebuilt trees freed along the way) gives the same results with
    torch's caching allocator as with the library's pool, and returns every
    block."""
    import torch

    import paper_2207_01834_amd._binding as pg
    init, rounds = datagen.bdl_rounds(50_000, 3, 20_000, 3_000, 3, seed=17)

    def run():
        B = pg.BDLTree(3, torch.int32, leaf=8, X=256, device=dev)
        B.insert(torch.from_numpy(init).to(dev))
        pool, outs = init, []
        for rd in rounds:
            B.insert(torch.from_numpy(rd["insert"]).to(dev))
            pool = np.concatenate([pool, rd["insert"]])
            E = datagen.choose_erase(pool, 15_000, rd["erase_seed"])
            outs.append(B.erase(torch.from_numpy(E).to(dev)))
            i, dd = B.knn(torch.from_numpy(rd["queries"]).to(dev), 6)
            torch.cuda.synchronize()
            outs.append((i.cpu().numpy(), dd.cpu().numpy()))
        outs.append(B.size())
        del B
        gc.collect()
        torch.cuda.synchronize()
        return outs

    ref = run()
    say("BDL sequence through torch's caching allocator")
    pg.use_torch_allocator(True)
    try:
        before = torch.cuda.memory_allocated(dev)
        got = run()
        assert torch.cuda.memory_allocated(dev) == before  # every block came back
    finally:
        pg.use_torch_allocator(False)
    for a, b in zip(ref, got):
        if isinstance(a, tuple):
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
        else:
            assert a == b


_CACHE_CHILD = r"""
import sys
sys.path.insert(0, sys.argv[1])
import numpy as np, torch
from paper_2207_01834_amd import _binding as pg, datagen
init, rounds = datagen.bdl_rounds(60_000, 3, 30_000, 5_000, 3, seed=23)
B = pg.BDLTree(3, torch.int32, leaf=8, X=512, device="cuda:0")
B.insert(torch.from_numpy(init).to("cuda:0"))
pool, h = init, []
for j, rd in enumerate(rounds):
    B.insert(torch.from_numpy(rd["insert"]).to("cuda:0"))
    pool = np.concatenate([pool, rd["insert"]])
    E = datagen.choose_erase(pool, 20_000, rd["erase_seed"])
    h.append(B.erase(torch.from_numpy(E).to("cuda:0")))
    if j == 1 and sys.argv[2] == "release":
        pg.release_cached()
    i, d = B.knn(torch.from_numpy(rd["queries"]).to("cuda:0"), 7)
    torch.cuda.synchronize()
    h.append(int(np.bitwise_xor.reduce(i.cpu().numpy().ravel() * 1000003 + d.cpu().numpy().ravel())))
h.append(B.size())
del B
pg.release_cached()
print(" ".join(str(v) for v in h))
"""


def test_block_cache_limits(dev):
    # the same BDL sequence with the default cache, with a 4 MiB limit (a
    # trim, with its device synchronisation, at nearly every large free) and
    # with an explicit release mid-sequence gives the same erase counts,
    # k-NN results and sizes
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

    def child(limit, mode):
        env = dict(os.environ)
        env.pop("PG_CACHE_LIMIT_MIB", None)
        if limit is not None:
            env["PG_CACHE_LIMIT_MIB"] = str(limit)
        say(f"block-cache child: limit {limit} MiB, {mode}")
        r = subprocess.run([sys.executable, "-c", _CACHE_CHILD, root, mode], env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stderr[-2000:]
        return r.stdout.strip().splitlines()[-1]

    a = child(None, "keep")
    assert child(4, "keep") == a
    assert child(None, "release") == a
