"""SCF iterations replayed from a captured HIP graph (options.graphs = 1)
against the same batch stepped with plain launches.

From the second iteration on the graph batch replays one captured
iteration.  Both batches are stepped in lockstep on their own streams with
eager torch work and host synchronisations between the steps; after every
step the energies, convergence measures, densities and active counts must
agree.  The kernels and their order are the same, only the J/K and XC
partial sums may add in another order (atomics, ~1e-15 relative per sum),
so FP64 energies and densities agree to 1e-9 and the mixed path (whose FP32
Fock matrix carries ~1e-7 relative noise into each step) to 1e-6.
"""
import numpy as np
import pytest

from paper_2311_01135_amd import molgen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def ks():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2311_01135_amd import ks as K
    K.load()
    return K


def _mols():
    return [molgen.water(0)] + [molgen.tree(n, 11, n) for n in (2, 3, 4, 5)]


@pytest.mark.parametrize("prec", [0, 1])
def test_graph_steps_equal_plain_steps(ks, prec):
    tol = 1e-9 if prec == 0 else 1e-6
    mols = _mols()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    print("graph vs plain, prec %d, %d molecules" % (prec, len(mols)), flush=True)
    with ks.Batch(mols, prec=prec, graphs=1, stream=s1.cuda_stream) as bg, \
            ks.Batch(mols, prec=prec, graphs=0, stream=s2.cuda_stream) as bp:
        scratch = torch.zeros(1 << 20, device="cuda")
        steps = 0
        prevE = [None] * len(mols)
        while True:
            ng = bg.scf_step()
            # eager work and synchronisations between the replays
            with torch.cuda.stream(s1):
                scratch.add_(1.0)
            torch.cuda.synchronize()
            npl = bp.scf_step()
            steps += 1
            assert ng == npl, (steps, ng, npl)
            for m in range(len(mols)):
                Eg, dEg, eg = bg.convergence(m)
                Ep, dEp, ep = bp.convergence(m)
                assert abs(Eg - Ep) <= tol, (steps, m, Eg, Ep)
                # dE is this iteration's energy minus the previous one's (the
                # first iteration compares with 0); a retired molecule keeps
                # the values of its last iteration
                if prevE[m] is not None and Ep != prevE[m][0]:
                    assert abs(dEp - (Ep - prevE[m][0])) <= 1e-12 * max(1.0, abs(Ep)), (steps, m, dEp, Ep, prevE[m])
                    assert abs(dEg - (Eg - prevE[m][1])) <= 1e-12 * max(1.0, abs(Eg)), (steps, m, dEg, Eg, prevE[m])
                elif prevE[m] is None:
                    assert dEp == Ep and dEg == Eg, (steps, m, dEp, Ep)
                prevE[m] = (Ep, Eg)
                assert abs(eg - ep) <= tol, (steps, m, eg, ep)
                assert np.abs(bg.matrix(m, "P") - bp.matrix(m, "P")).max() <= tol, (steps, m)
            if ng == 0:
                break
            assert steps < 60
        assert steps >= 3          # at least two replays of the captured iteration
        assert float(scratch[0]) == steps
        for m in range(len(mols)):
            rg, rp = bg.result(m), bp.result(m)
            assert rg["status"] == rp["status"] == 1
            assert rg["n_iter"] == rp["n_iter"]
            assert abs(rg["E"] - rp["E"]) <= tol
            assert abs(rg["gap"] - rp["gap"]) <= tol


def test_graph_option_validation(ks):
    with pytest.raises(ks.KsError):
        ks.Batch([molgen.water(0)], graphs=2)
