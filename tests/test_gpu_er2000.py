"""The correlated ER workload at n = 2000 (p = 0.01, rho = 0.8, barycenter
start, eps = 0.03 max|G|, Sinkhorn tolerance 1e-6 with at most 1000
iterations, at most 30 FW iterations) end to end: the device solver in fp32
against the FP64 oracle run on the same pair. Same number of FW iterations
and the same step sequence, Sinkhorn iteration counts within one sweep, the
relaxed objective within 1e-5 relative, and match ratios within 0.005 of
each other."""
import time

import numpy as np
import pytest

from oracle import goat_oracle as O
from paper_2111_05366_amd import inputs as I

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def G():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2111_05366_amd import goat
    goat.lib()
    yield goat
    goat.release_workspace()


@pytest.mark.parametrize("lap", [0, 1])
def test_er2000_end_to_end(G, lap):
    g = I.workload_er_2000()
    A = torch.as_tensor(g.A, device="cuda")
    B = torch.as_tensor(g.B, device="cuda")
    t0 = time.perf_counter()
    r = G.solve(A, B, prec="fp32", sk_max=1000, fw_max=30, lap=lap)
    t_gpu = time.perf_counter() - t0
    t0 = time.perf_counter()
    ref = O.goat(g.A, g.B, opt=O.GoatOptions(sk_max=1000, fw_max=30), record=True)
    t_orc = time.perf_counter() - t0
    mg = float(np.mean(r.perm == g.truth))
    mo = O.match_ratio(ref.perm, g.truth)
    st = r.stats
    print(f"n=2000 ER: device {st.fw_iters} FW iterations, {st.ms_loop:.1f} ms loop "
          f"({st.fw_iters / (st.ms_loop * 1e-3):.1f} FW it/s), Sinkhorn {[h['sk_iters'] for h in r.history]}, "
          f"assignment {st.ms_lap:.1f} ms ({'device' if st.lap_device else 'host'}), total {t_gpu:.2f} s; "
          f"oracle {ref.fw_iters} FW iterations, Sinkhorn {[h['sk_iters'] for h in ref.history]}, {t_orc:.1f} s; "
          f"match ratio {mg:.4f} vs {mo:.4f}")
    assert st.fw_iters == ref.fw_iters
    for h, o in zip(r.history, ref.history):
        assert h["t"] == pytest.approx(o["t"], abs=1e-4)
        # The stop rule is tested after every sweep on both sides. The
        # device's row-marginal error differs from the FP64 one by at most
        # its compensated-potential floor (about 2.4e-7 at n = 10,000, less
        # here), so a solve whose error crosses the 1e-6 tolerance within
        # that band can stop one sweep earlier or later.
        assert abs(h["sk_iters"] - o["sk_iters"]) <= 1
        assert h["fP"] == pytest.approx(o["fP"], rel=1e-5)
        assert h["c"] == pytest.approx(o["c"], rel=1e-5)
    f_ref = O.relaxed_objective(g.A.astype(np.float64), g.B.astype(np.float64), ref.P)
    print(f"final objective {st.f_final!r} vs oracle {f_ref!r}: rel {abs(st.f_final - f_ref) / abs(f_ref):.2e}")
    assert st.f_final == pytest.approx(f_ref, rel=1e-5)
    assert abs(mg - mo) <= 0.005
