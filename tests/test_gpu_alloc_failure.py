"""Device allocation failures: the library reports NUFFT2_ERR_ALLOC, frees
whatever it had allocated, and keeps working once memory is available again.

The failures are forced from the host: by a plan larger than the device's
memory, and by holding nearly all device memory in torch tensors while a
request runs through the serving loop.  No kernel is involved in a failure.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

MiB = 1 << 20
GiB = 1 << 30


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2605_01313_amd import nufft2  # noqa: F401  (fails loudly if not built)
    return torch, torch.device("cuda:0")


def device_free(torch):
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return torch.cuda.mem_get_info()[0]


def test_plan_larger_than_the_device_fails_and_frees_its_workspaces(torch_dev):
    """FP64, 2047 x 2047 modes, 1000 fields: the theta-pass buffer (134 GB)
    fits, the fine grids (268 GB) do not; the plan fails with ERR_ALLOC and
    the device's free memory is what it was before."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import nufft2
    say("case plan_too_large fp64 K=2047 F=1000")
    free0 = device_free(torch)
    st, h = nufft2.nufft2_plan(nufft2.NUFFT2_FP64, 2047, 2047, 1000, 1e-12, None,
                               torch.cuda.current_stream().cuda_stream)
    assert st == nufft2.NUFFT2_ERR_ALLOC, nufft2.nufft2_strerror(st)
    assert not h.value
    free1 = device_free(torch)
    say(f"  free before {free0 / GiB:.3f} GiB, after {free1 / GiB:.3f} GiB")
    assert abs(free1 - free0) <= 2 * MiB
    # a normal plan still works afterwards
    from paper_2605_01313_amd import Plan
    p = Plan("fp64", 31, 31, n_fields=1, eps=1e-12)
    phi = torch.linspace(0, 6, 100, dtype=torch.float64, device=dev)
    p.setpts(phi, phi * 0.5)
    out = p.exec(torch.ones((1, 31, 31), dtype=torch.complex128, device=dev))
    torch.cuda.synchronize()
    assert torch.isfinite(out.real).all()
    p.destroy()


def big_request(torch, rng, J, F):
    K = 2 * J - 1
    c = synth.random_complex(rng, (F, K, K)) * synth.envelope_algebraic(K, K, 1.5)[None]
    n = 4096
    phi = rng.uniform(0, 2 * np.pi, n)
    theta = rng.uniform(0, np.pi, n)
    return (torch.from_numpy(c).to(torch.complex64).pin_memory(), torch.from_numpy(phi).pin_memory(),
            torch.from_numpy(theta).pin_memory())


def test_server_request_fails_while_the_device_is_full_then_succeeds(torch_dev):
    """With all but about 512 MiB of device memory held by torch, a request
    whose plan needs about 600 MB fails with ERR_ALLOC, keeping only its
    slot's input/output buffer, while a small one beside it completes; once
    the memory is released the same large request completes.  A second
    server afterwards, warmed up the same way, finds the device memory the
    first one found (nothing left behind)."""
    torch, dev = torch_dev
    from paper_2605_01313_amd import Server, nufft2
    say("case server_device_full")
    rng = np.random.default_rng(5)
    big = big_request(torch, rng, 1024, 3)
    small = big_request(torch, rng, 32, 1)
    slot_bytes = (big[0].numel() * 8 + 2 * 8 * big[1].numel() + 3 * 8 * big[1].numel() + MiB - 1) // MiB * MiB

    def warmed_server():
        # streams, events and a small cached plan exist and have run once
        srv = Server(hbm_budget=1024 * GiB, max_inflight=2)
        st, _ = srv.wait(srv.submit("fp32", *small, 1e-6))
        assert st == nufft2.NUFFT2_OK
        return srv, device_free(torch)

    srv, free_w = warmed_server()
    hold = []
    free = torch.cuda.mem_get_info()[0]
    while free > 768 * MiB:
        take = min(8 * GiB, free - 512 * MiB)
        hold.append(torch.empty(take, dtype=torch.uint8, device=dev))
        free = torch.cuda.mem_get_info()[0]
    torch.cuda.synchronize()
    free_a = torch.cuda.mem_get_info()[0]
    say(f"  holding {sum(h.numel() for h in hold) / GiB:.1f} GiB, {free_a / MiB:.0f} MiB free")
    st_big, _ = srv.wait(srv.submit("fp32", *big, 1e-6))
    free_b = torch.cuda.mem_get_info()[0]
    st_small, _ = srv.wait(srv.submit("fp32", *small, 1e-6))
    say(f"  while full: large request status {st_big} (kept {(free_a - free_b) / MiB:.0f} MiB, slot buffer "
        f"{slot_bytes / MiB:.0f} MiB), small request status {st_small}")
    assert st_big == nufft2.NUFFT2_ERR_ALLOC
    assert st_small == nufft2.NUFFT2_OK
    # the failed plan's workspaces were freed: only the slot's buffer stays
    assert free_a - free_b <= slot_bytes + 16 * MiB
    del hold
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    st_big, _ = srv.wait(srv.submit("fp32", *big, 1e-6))
    say(f"  after release: large request status {st_big}")
    assert st_big == nufft2.NUFFT2_OK
    s = srv.stats()
    assert s["failed"] == 1 and s["completed"] == 3
    srv.destroy()
    srv2, free_w2 = warmed_server()
    srv2.destroy()
    say(f"  free with a warmed server: first {free_w / GiB:.3f} GiB, second {free_w2 / GiB:.3f} GiB")
    assert abs(free_w2 - free_w) <= 16 * MiB
