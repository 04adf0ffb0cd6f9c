"""HIP-graph capture of a chemistry flow step: the integrator and the
surrogate-with-fallback calls enqueue no allocation, host synchronisation or
memset, so a captured step replays.  Each replay is checked bitwise against
the eager result, with eager work of the program between replays."""
import numpy as np
import pytest

from test_gpu_integrate import _say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


def _dev(torch, a, dtype=None):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype or torch.float64, device="cuda:0")


def _replay_check(torch, g, outs, ref, eager_between):
    for rep in range(3):
        g.replay()
        torch.cuda.synchronize()
        for o, r in zip(outs, ref):
            assert torch.equal(o, r), f"replay {rep} differs from the eager step"
        eager_between()
        torch.cuda.synchronize()


def test_graph_captured_integrator_step(torch, mech_dir):
    from chemgen.fields import cells4096
    from chemgen.mechanism import read_mechanism
    from paper_2312_13513_amd import chem
    mpy = read_mechanism(str(mech_dir / "M9.mech"))
    f = cells4096(mpy, n=2048, seed=9)
    mech = chem.Mechanism(str(mech_dir / "M9.mech"), 0)
    T0, p, Y0 = _dev(torch, f.T), _dev(torch, f.p), _dev(torch, f.Y)
    T, Y = T0.clone(), Y0.clone()
    st = torch.zeros(f.n, dtype=torch.int32, device="cuda:0")
    # eager reference
    mech.integrate(T, p, Y, f.dt, status=st)
    torch.cuda.synchronize()
    ref = (T.clone(), Y.clone(), st.clone())
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        T.copy_(T0)
        Y.copy_(Y0)
        mech.integrate(T, p, Y, f.dt, status=st)   # warm-up on the capture stream
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            T.copy_(T0)
            Y.copy_(Y0)
            mech.integrate(T, p, Y, f.dt, status=st)
    torch.cuda.synchronize()
    other_T, other_Y = T0.clone(), Y0.clone()

    def eager():
        other_T.copy_(T0)
        other_Y.copy_(Y0)
        mech.integrate(other_T, p, other_Y, f.dt)
        T.fill_(0.0)
        Y.fill_(0.0)
        st.fill_(-1)

    _replay_check(torch, g, (T, Y, st), ref, eager)
    assert torch.equal(other_T, ref[0])
    _say("[graph] integrator step: 3 replays equal to the eager step")
    mech.close()


def test_graph_captured_surrogate_step(torch, mech_dir):
    from chemgen.fields import zones128
    from chemgen.mechanism import read_mechanism
    from chemgen.surrogate_data import init_params, network_dims
    from oracle import surrogate as S
    from paper_2312_13513_amd import chem
    mpy = read_mechanism(str(mech_dir / "M35.mech"))
    f = zones128(mpy, shape=(8, 8, 16))
    K = mpy.K
    mech = chem.Mechanism(str(mech_dir / "M35.mech"), 0)
    surr = chem.Surrogate(mech, 64, 64, 64)
    surr.set_params(init_params(network_dims(K, 64, 64, 64), 3))
    raw = S.features(f.T, f.p, f.Y)
    rng = np.random.default_rng(4)
    surr.set_norm(np.concatenate([raw.mean(0), raw.std(0), np.zeros(K), rng.uniform(1e-10, 1e-9, K), [f.dt]]))
    checks = chem.chem_surrogate_default_checks()
    checks.T_in_max = 1500.0     # hot cells go to the integrator, the others to the network
    T0, p, Y0 = _dev(torch, f.T), _dev(torch, f.p), _dev(torch, f.Y)
    T, Y = T0.clone(), Y0.clone()
    mask = torch.zeros(f.n, dtype=torch.int32, device="cuda:0")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    surr.infer(T, p, Y, f.dt, checks=checks, mask=mask, fallback_count=cnt)
    torch.cuda.synchronize()
    ref = (T.clone(), Y.clone(), mask.clone(), cnt.clone())
    _say(f"[graph] surrogate step: fallback {int(cnt.item())} of {f.n} cells")
    assert 0 < int(cnt.item()) < f.n          # both the network and the integrator take part
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        T.copy_(T0)
        Y.copy_(Y0)
        surr.infer(T, p, Y, f.dt, checks=checks, mask=mask, fallback_count=cnt, stream=s)
        s.synchronize()
        with torch.cuda.graph(g, stream=s):
            T.copy_(T0)
            Y.copy_(Y0)
            surr.infer(T, p, Y, f.dt, checks=checks, mask=mask, fallback_count=cnt, stream=s)
    torch.cuda.synchronize()

    def eager():
        T.fill_(0.0)
        Y.fill_(0.0)
        mask.fill_(7)
        cnt.fill_(-3)
        mech.integrate(_dev(torch, f.T), p, _dev(torch, f.Y), f.dt)

    _replay_check(torch, g, (T, Y, mask, cnt), ref, eager)
    surr.close()
    mech.close()
