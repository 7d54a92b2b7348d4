"""GPU tests of the request server (continuous batching) through the C ABI.

Each request's output must be the same served alone and served in a mix of
concurrent requests under a tight memory budget -- bit for bit, for u8 and for
f32 -- and equal to the single-image call and, on u8, to the oracle."""
from __future__ import annotations

import numpy as np
import pytest

import oracle
from paper_2505_12425_amd import workloads as wl
from tests.gpu_util import assert_u8_equal, say

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

from paper_2505_12425_amd import kr  # noqa: E402


def _fetch(ptr, nbytes, shape, dtype):
    """Copy an arena output (device pointer) into a host array."""
    t = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    kr.check(kr.lib().kr_hbm_copy(t.data_ptr(), ptr, nbytes, kr._stream(None)))
    torch.cuda.synchronize()
    return t.cpu().numpy().view(dtype).reshape(shape)


def _requests(rng, n, c):
    reqs = []
    for i in range(n):
        h, w = int(rng.integers(30, 900)), int(rng.integers(30, 900))
        im = wl.uniform_u8(h, w, c, seed=500 + i)
        t = int(rng.choice([16, 50, 224, 300]))
        if i % 3 == 2:
            m = wl.affine_compose(h, w, rng.uniform(-45, 45), t / max(h, w) * rng.uniform(0.5, 1.5),
                                  rng.uniform(-0.2, 0.2), (t - w) / 2.0, (t - h) / 2.0)
            reqs.append(("warp", im, t, m))
        else:
            reqs.append(("resize", im, t, None))
    return reqs


def _serve(reqs, srcs, c, out, budget, slots, max_batch):
    srv = kr.Server(budget, slots=slots, max_batch=max_batch, c=c, out=out, border=kr.REPLICATE)
    dt = np.uint8 if out == "u8" else np.float32
    ids = {}
    for (op, im, t, m), s in zip(reqs, srcs):
        ids[srv.submit(kr.make_request(op, s, t, t, m))] = (t, len(ids))
    results = [None] * len(reqs)
    spins = 0
    while any(r is None for r in results):
        for rid, ptr, nbytes, _t in srv.poll():
            t, k = ids[rid]
            results[k] = _fetch(ptr, nbytes, (t, t, c), dt)
            srv.release(rid)
        spins += 1
        assert spins < 10_000_000
    used, queued, busy = srv.stats()
    assert used == 0 and queued == 0 and busy == 0
    srv.close()
    return results


@pytest.mark.parametrize("c,out", [(3, "u8"), (3, "f32"), (4, "u8"), (1, "u8"), (2, "f32")])
def test_served_alone_equals_served_in_mix(c, out):
    rng = np.random.default_rng(11 + c)
    reqs = _requests(rng, 30, c)
    srcs = [torch.from_numpy(im).cuda() for _, im, _, _ in reqs]
    say(f"serve mix c={c} out={out}: 30 requests")
    esize = 1 if out == "u8" else 4
    biggest = max(t * t * c * esize for _, _, t, _ in reqs)
    # tight budget: a few outputs at a time -> requests queue for memory
    mixed = _serve(reqs, srcs, c, out, budget=3 * biggest + 4096, slots=3, max_batch=4)
    alone = [_serve([r], [s], c, out, budget=biggest + 4096, slots=1, max_batch=1)[0]
             for r, s in zip(reqs, srcs)]
    dt = torch.uint8 if out == "u8" else torch.float32
    for k, ((op, im, t, m), s) in enumerate(zip(reqs, srcs)):
        assert np.array_equal(mixed[k], alone[k]), f"request {k}: mix != alone"
        single = torch.empty((t, t, c), dtype=dt, device="cuda")
        if op == "warp":
            kr.warp_affine(s, single, m, border=kr.REPLICATE)
        else:
            kr.resize(s, single, border=kr.REPLICATE)
        torch.cuda.synchronize()
        assert np.array_equal(single.cpu().numpy(), mixed[k]), f"request {k}: served != single call"
        if out == "u8" and k % 5 == 0:
            exp = (oracle.warp(im, m, t, t, "u8", border=oracle.REPLICATE) if op == "warp"
                   else oracle.resize(im, t, t, "u8", oracle.REPLICATE))
            assert_u8_equal(mixed[k], exp, f"request {k} vs oracle")


def test_run_trace_and_budget():
    rng = np.random.default_rng(5)
    reqs = _requests(rng, 40, 3)
    srcs = [torch.from_numpy(im).cuda() for _, im, _, _ in reqs]
    krs = [kr.make_request(op, s, t, t, m) for (op, _, t, m), s in zip(reqs, srcs)]
    arrivals = np.cumsum(rng.exponential(20e-6, size=len(krs)))
    say("serve trace 40 requests")
    srv = kr.Server(8 << 20, slots=4, max_batch=8, c=3, out="u8")
    lat = srv.run_trace(krs, arrivals)
    assert all(v > 0 for v in lat), lat
    assert srv.stats() == (0, 0, 0)
    with pytest.raises(kr.KrError) as e:
        srv.submit(kr.make_request("resize", srcs[0], 4000, 4000))
    assert e.value.status == kr.ERR_OUT_OF_BUDGET
    srv.close()
