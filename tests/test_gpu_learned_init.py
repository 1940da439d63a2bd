"""The learned FFCP initializer against the method without it.

Cores come from the pipeline itself: seeded 300^3 CP tensors of rank 20
with per-mode column congruence U[0.5, 0.95] and SNR U[20, 40] dB, compressed
by rt_tucker_rand in the precision form (BF16, two sweeps) to 20^3 cores.
The network is trained on the GPU by rt_mlp_train_step; on held-out cores
FFCP-ALS (tol 1e-6) starts from the network's factors (guarded by the HOSVD
start) and from the HOSVD start alone.  The test asserts what the paper's
initialization cannot give: fewer ALS iterations on average, with a final
fit no worse on every core (the guard keeps the HOSVD start when the
network's is worse).
"""

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

I, R, RT = 300, 20, 30


@pytest.fixture(scope="module")
def P():
    import paper_1412_1885_amd as P
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    P.lib()
    return P


def pipeline_cores(P, k0, count):
    dev = torch.device("cuda")
    Gs, Us = [], []
    for k in range(k0, k0 + count):
        snr = synth.rngs((5, k))["noise"].uniform(20.0, 40.0)
        d = synth.cp_congruent_device((5, k), (I, I, I), R, 0.5, 0.95, snr, (RT,) * 3,
                                      sweeps=2, device=dev)
        om = [torch.from_numpy(o).to(dev) for o in synth.f32(d["omegas"])]
        omt = [[torch.from_numpy(o).to(dev) for o in synth.f32(lst)]
               for lst in d["omega_tildes"]]
        out = P.tucker_rand(d["Y"], om, omt, ranks=(R, R, R), sweeps=2, precision="bf16",
                            sync=False)
        Gs.append(out["G"])
        Us.append(out["U"])
    torch.cuda.synchronize()
    return torch.stack(Gs), Us


def test_learned_init_needs_fewer_als_iterations(P):
    Gtr, _ = pipeline_cores(P, 0, 1024)
    Gev, Uev = pipeline_cores(P, 100000, 24)
    net = P.MLP((R, R, R), R, (1024, 1024))
    W, b = synth.mlp_weights(77, net.dims)
    W[2] = W[2] * 0.1
    net.load(W, b)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    losses = []
    for ep in range(24):
        perm = torch.randperm(Gtr.shape[0], device="cuda", generator=gen)
        lr = 1e-3 * 0.5 ** (ep // 6)
        for i in range(0, Gtr.shape[0], 256):
            losses.append(float(net.train_step(Gtr[perm[i:i + 256]].contiguous(), lr).mean()))
    assert losses[-1] < 0.1 * losses[0]          # the network learned the cores
    Vs = net.split(net.forward(Gev))
    it_h, it_l, fit_h, fit_l = [], [], [], []
    for k in range(Gev.shape[0]):
        G = Gev[k].contiguous()
        h = P.ffcp(Uev[k], G, R, update="als", init="hosvd", max_it=1000, tol=1e-6)
        l = P.ffcp(Uev[k], G, R, update="als", init="coeff_guarded",
                   A_init=[v[k].contiguous() for v in Vs], max_it=1000, tol=1e-6)
        it_h.append(int(h["info"]["iterations"]))
        it_l.append(int(l["info"]["iterations"]))
        fit_h.append(float(h["info"]["fit"]))
        fit_l.append(float(l["info"]["fit"]))
    it_h, it_l = np.array(it_h), np.array(it_l)
    print(f"ALS iterations: HOSVD start {it_h.mean():.1f}, learned start {it_l.mean():.1f}")
    assert it_l.mean() < 0.8 * it_h.mean()
    assert np.all(np.array(fit_l) >= np.array(fit_h) - 1e-4)
