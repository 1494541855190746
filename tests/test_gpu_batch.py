"""Batched diagrams (many grids in one pipeline run) against the same grids
computed alone and against the oracle: equal bit for bit, per item, in the
order dms_diagram returns. Also the captured-graph replay of the order and
gradient kernels, and the error path of an item wider than the cross-section.
"""
import numpy as np
import pytest

import oracle
import synthfields as sf


def _fields(rng, n, lo, hi):
    out = []
    for i in range(n):
        shape = tuple(int(x) for x in rng.integers(lo, hi, size=3))
        seed = int(rng.integers(0, 1 << 30))
        if i % 3 == 0:
            out.append(sf.noise(shape, seed))
        else:
            out.append(sf.gaussians(shape, seed, k=int(rng.integers(1, 8)), noise_frac=0.01))
    return out


def _same(a, b):
    return all(np.array_equal(a[d].cpu().numpy(), b[d].cpu().numpy()) for d in range(3))


@pytest.mark.gpu
def test_batch_equals_alone_and_oracle():
    import torch
    from paper_2206_13932_amd import dms
    ctx = dms.Context(0)
    fs = _fields(np.random.default_rng(1), 24, 3, 28)
    dev = [torch.from_numpy(f).cuda() for f in fs]
    got = ctx.diagram_batch(dev)
    info = ctx.batch_info()
    print(f"[batch] super grid {info[:3]}, real vertices {info[3]}", flush=True)
    for i, f in enumerate(fs):
        res = oracle.run(f)
        for d in range(3):
            assert np.array_equal(got[i][d].cpu().numpy(), res.pairs[d]), (i, f.shape, d)
        assert _same(got[i], ctx.diagram(dev[i])), i
    ctx.close()


@pytest.mark.gpu
def test_batch_with_infinities():
    """Items holding +inf (a whole box face, so real +inf vertices touch the
    separators) and -inf: batched = alone = oracle. Separators are ordered
    above every real value, +inf included."""
    import torch
    from paper_2206_13932_amd import dms
    ctx = dms.Context(0)
    rng = np.random.default_rng(11)
    fs = [sf.with_infinities(f, 100 + i, 0.05 + 0.05 * (i % 4), 0.05) for i, f in enumerate(_fields(rng, 12, 3, 20))]
    dev = [torch.from_numpy(f).cuda() for f in fs]
    got = ctx.diagram_batch(dev)
    for i, f in enumerate(fs):
        print(f"[batch-inf] item={i} shape={f.shape}", flush=True)
        res = oracle.run(f)
        for d in range(3):
            assert np.array_equal(got[i][d].cpu().numpy(), res.pairs[d]), (i, f.shape, d)
        assert _same(got[i], ctx.diagram(dev[i])), i
    ctx.close()


@pytest.mark.gpu
def test_batch_of_one_and_mixed_sizes():
    import torch
    from paper_2206_13932_amd import dms
    ctx = dms.Context(0)
    fs = _fields(np.random.default_rng(2), 48, 16, 65)
    dev = [torch.from_numpy(f).cuda() for f in fs]
    got = ctx.diagram_batch(dev)
    for i in range(len(fs)):
        assert _same(got[i], ctx.diagram(dev[i])), i
    one = ctx.diagram_batch(dev[:1])
    assert _same(one[0], got[0])
    ctx.close()


@pytest.mark.gpu
def test_batch_graph_replay():
    import torch
    from paper_2206_13932_amd import dms
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        ctx = dms.Context(0, stream=stream)
        rng = np.random.default_rng(3)
        shapes = [tuple(int(x) for x in rng.integers(8, 40, size=3)) for _ in range(16)]
        for rep in range(3):
            fs = [sf.gaussians(s, 1000 * rep + j, k=4, noise_frac=0.01) for j, s in enumerate(shapes)]
            dev = [torch.from_numpy(f).cuda() for f in fs]
            g = ctx.diagram_batch(dev, use_graph=True)
            plain = ctx.diagram_batch(dev, use_graph=False)
            for i in range(len(fs)):
                assert _same(g[i], plain[i]), (rep, i)
                assert _same(g[i], ctx.diagram(dev[i])), (rep, i)
        info = ctx.batch_info()
        print(f"[batch] graph launches {info[4]}, captures {info[5]}, plain runs {info[6]}", flush=True)
        assert info[5] == 1 and info[4] >= 3  # a capacity retry replays it again
        ctx.close()
    torch.cuda.synchronize()


@pytest.mark.gpu
def test_batch_rejects_wide_items():
    import torch
    from paper_2206_13932_amd import dms
    ctx = dms.Context(0)
    f = torch.from_numpy(sf.noise((8, 8, 40), 0)).cuda()
    with pytest.raises(dms.DmsError):
        ctx.diagram_batch([f], cross=(32, 32))
    # the context stays usable
    assert _same(ctx.diagram_batch([f])[0], ctx.diagram(f))
    ctx.close()
