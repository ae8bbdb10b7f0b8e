"""AR(1) coupling scenarios (Table 1, eq. 12-16) through the delay scan (eq. 5) at full size:
50 trials x 3000 samples, windows of 300 samples (N = 15 000), 500 surrogates, k = 4.

Where the coupling is on, the scan must find significant transfer at the simulated delay;
where it is off, the estimates stay near zero.  A seeded sample of chunks is checked against
the oracle at the same tolerance as every other parity test.
"""
import sys

import numpy as np
import pytest

import synth
from oracle import oracle

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def te():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1401_4068_amd as te
    te.lib()
    return te


def _scan(te, scenario):
    import torch
    wl = synth.ar_scenarios(scenario)
    x = torch.from_numpy(wl.x).cuda()
    y = torch.from_numpy(wl.y).cuda()
    perms = torch.from_numpy(wl.perms).cuda()
    plan = te.Plan.from_workload(wl)
    u_values = wl.meta["u_values"]
    te_scan, u_best, te_surr, pv = plan.delay_scan(x, y, u_values, perms)
    for p in range(wl.n_pairs):
        say(wl.meta["directions"][p], u_best[p].tolist(), np.round(te_scan[p].max(axis=1), 4).tolist(),
            pv[p].tolist())
    return wl, u_values, te_scan, u_best, te_surr, pv


def test_ar_unidirectional_delay_and_significance(te):
    wl, u_values, te_scan, u_best, te_surr, pv = _scan(te, 1)
    XY, YX = 0, 1
    # coupling fully on in the window 1100-1400: delay 10 found, no surrogate reaches it
    assert u_best[XY, 3] == 10 and pv[XY, 3] == 0.0
    # coupling off before 800: near-zero transfer; no coupling from Y to X at all
    assert np.all(te_scan[XY, :2].max(axis=1) < 0.03)
    assert np.all(te_scan[YX].max(axis=1) < 0.03)
    # oracle on a seeded sample: two originals and two surrogates at the chosen delay
    jobs = [(XY, 1100, 300, 50, -1), (YX, 200, 300, 50, -1)]
    ref = oracle.te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, 10, wl.k, jobs, wl.perms)
    assert abs(ref[0] - te_scan[XY, 3, u_values.index(10)]) <= 1e-9
    assert abs(ref[1] - te_scan[YX, 0, u_values.index(10)]) <= 1e-9
    rows = [(XY * wl.n_points + 3) * wl.n_surrogates + s for s in (0, 499)]
    sj = [(XY, 1100, 300, 50, r) for r in rows]
    sref = oracle.te_jobs(wl.x, wl.y, wl.d_y, wl.d_x, wl.tau, 10, wl.k, sj, wl.perms)
    assert abs(sref[0] - te_surr[XY, 3, 0]) <= 1e-9 and abs(sref[1] - te_surr[XY, 3, 499]) <= 1e-9


def test_ar_bidirectional_delays(te):
    wl, u_values, te_scan, u_best, te_surr, pv = _scan(te, 3)
    XY, YX = 0, 1
    # last window (2300-2600): both couplings on, X -> Y at delay 10 and Y -> X at delay 20
    assert u_best[XY, 7] == 10 and pv[XY, 7] == 0.0
    assert u_best[YX, 7] == 20 and pv[YX, 7] == 0.0
    # before the first onset (windows starting at 200 and 500) neither direction carries transfer
    assert np.all(te_scan[:, :2].max(axis=2) < 0.03)


def test_delay_recovery_against_amount_of_data(te):
    """The robustness evaluation on AR data: with enough pooled points (M >= 10 000) the scan
    recovers the coupling delay of 10 samples and the surrogate test rejects independence."""
    import torch
    wl = synth.ar_robustness()
    x = torch.from_numpy(wl.x).cuda()
    y = torch.from_numpy(wl.y).cuda()
    perms = torch.from_numpy(wl.perms).cuda()
    te_scan, u_best, _, pv = te.Plan.from_workload(wl).delay_scan(x, y, wl.meta["u_values"], perms)
    say("M", wl.meta["points"], "u_best", u_best[0].tolist(), "p", pv[0].tolist())
    for c, m in enumerate(wl.meta["points"]):
        if m >= 10000:
            assert u_best[0, c] == 10 and pv[0, c] == 0.0
