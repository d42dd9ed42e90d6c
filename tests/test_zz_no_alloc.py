"""pm_observe_time_noalloc (the forward map of Algorithm 1 without device
allocation) against pm_observe_time, through the C ABI.

Both entry points run the same kernels on the same Philox streams, so the
results must agree bit for bit: means, variances and endpoints.  Each case
makes two no-allocation calls in a row, the second with a smaller input, so
the second reads a scratch array that still holds the first call's contents.
The main-workload case uses the full 49 x 1e5 particle ensemble of the
torus benchmark (76,587 chunks, 78 MB of final states), which must fit the
fixed scratch, and checks that the device's free memory does not move across
the call.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def pm():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1808_10580_amd as pm
    pm.lib()
    return pm


def _pair(pm, prob_a, prob_n, u, obs, kappa, T, dt, np_, seed, endpoints):
    """Both entry points on the same input; returns the no-allocation means
    and the device's free memory just before and just after that call (all
    tensors of the test are allocated outside that window)."""
    import torch
    ma, va, *ea = prob_a.observe_time(u, obs, kappa, T, dt, np_, seed, endpoints=endpoints)
    assert prob_a.ctx.sync() == pm.PM_OK
    n_obs = obs.shape[0]
    mn = torch.full((n_obs,), float("nan"), dtype=torch.float64, device="cuda")
    vn = torch.full_like(mn, float("nan"))
    en = (torch.full((n_obs, np_, 2), float("nan"), dtype=torch.float64, device="cuda") if endpoints else None)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    prob_n.observe_time_noalloc(u, obs, kappa, T, dt, np_, seed, mn, vn, en)
    assert prob_n.ctx.sync() == pm.PM_OK
    free1 = torch.cuda.mem_get_info()[0]
    print(f"n_obs={n_obs} Np={np_} steps={round(T / dt)}: means equal {torch.equal(ma, mn)}, "
          f"free memory {free0} -> {free1}")
    assert torch.equal(ma, mn) and torch.equal(va, vn)
    if endpoints:
        assert torch.equal(ea[0], en)
    return mn, free0, free1


@pytest.mark.parametrize("engine", ["auto", "valu"])
def test_main_workload_twice_bitwise_and_no_allocation(pm, engine):
    import torch
    import workloads as W
    wl = W.time_main()
    ca, cn = pm.Context(0), pm.Context(0)
    for c in (ca, cn):
        c.set_velocity_engine(engine)
    pa = pm.Problem(ca, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    pn = pm.Problem(cn, "torus", wl.modes, theta0=wl.theta0, prec="fp32")
    u = torch.tensor(wl.u, dtype=torch.float64, device="cuda")
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    T = 20 * wl.dt
    # warm the kernels on the allocating context
    pa.observe_time(u, obs, wl.kappa, T, wl.dt, wl.n_particles, wl.seed)
    assert ca.sync() == pm.PM_OK
    m1, free0, free1 = _pair(pm, pa, pn, u, obs, wl.kappa, T, wl.dt, wl.n_particles, wl.seed, False)
    # a call that allocated its 78 MB of final states would show here
    assert free0 - free1 < (8 << 20), (free0, free1)
    assert np.all(np.isfinite(m1.cpu().numpy()))
    # second call, smaller: 7 points x 100 particles, 15 steps, with endpoints
    _pair(pm, pa, pn, u, obs[::7].contiguous(), wl.kappa, 15 * wl.dt, wl.dt, 100, wl.seed + 1, True)
    pa.close(); pn.close(); ca.close(); cn.close()


def test_fp64_twice_bitwise_and_context_buffers_intact(pm):
    import torch
    import workloads as W
    wl = W.time_small()
    ca, cn = pm.Context(0), pm.Context(0)
    pa = pm.Problem(ca, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    pn = pm.Problem(cn, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    u = torch.tensor(wl.u, dtype=torch.float64, device="cuda")
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    # the no-allocation context first allocates its own buffers in an ordinary call
    m0, v0 = pn.observe_time(u, obs, wl.kappa, wl.T, wl.dt, 300, wl.seed)
    assert cn.sync() == pm.PM_OK
    _pair(pm, pa, pn, u, obs, wl.kappa, wl.T, wl.dt, 1000, wl.seed, True)
    _pair(pm, pa, pn, u, obs[:2].contiguous(), wl.kappa, 10 * wl.dt, wl.dt, 65, wl.seed + 5, True)
    # the context's own buffers are back in place for its ordinary calls
    m2, v2 = pn.observe_time(u, obs, wl.kappa, wl.T, wl.dt, 300, wl.seed)
    assert cn.sync() == pm.PM_OK
    assert torch.equal(m0, m2) and torch.equal(v0, v2)
    pa.close(); pn.close(); ca.close(); cn.close()


def test_requests_beyond_the_scratch_are_rejected_before_launch(pm):
    import torch
    import workloads as W
    wl = W.time_small()
    c = pm.Context(0)
    p = pm.Problem(c, "torus", wl.modes, theta0=wl.theta0, prec="fp64")
    u = torch.tensor(wl.u, dtype=torch.float64, device="cuda")
    obs = torch.tensor(wl.obs, dtype=torch.float64, device="cuda")
    m = torch.full((obs.shape[0],), 7.0, dtype=torch.float64, device="cuda")
    v = torch.full_like(m, 7.0)
    np_max = pm.NOALLOC_MAX_CHUNKS // obs.shape[0] * 64
    with pytest.raises(pm.PMError) as e:
        p.observe_time_noalloc(u, obs, wl.kappa, wl.T, wl.dt, np_max + 1, wl.seed, m, v)
    assert e.value.status == pm.PM_EINVAL
    assert c.sync() == pm.PM_OK
    assert torch.all(m == 7.0) and torch.all(v == 7.0)  # nothing was launched
    p.close(); c.close()
