"""The learned FFCP initializer against the method without it.

Cores come from the pipeline itself: seeded 300^3 CP tensors of rank 20
with per-mode column congruence U[0.5, 0.95] and SNR U[20, 40] dB, compressed
by rt_tucker_rand in the precision form (BF16, two sweeps) to 20^3 cores.
The network is trained on the GPU by rt_mlp_train_step on 8192 such cores;
on 512 held-out cores FFCP-ALS (tol 1e-6) starts from the network's factors
(guarded by the HOSVD start), from the HOSVD start alone and from seeded
random factors.  The test asserts fewer ALS iterations than from the HOSVD
start on average and no more than about a random start's, with final fits
as good as the HOSVD start's over the set (the guard keeps the HOSVD start
when the network's initial fit is worse).
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
    """8192 training cores and 512 held-out ones; on each held-out core
    FFCP-ALS to a fit change below 1e-6 from three starts: seeded N(0,1)
    factors, the HOSVD start of the core, and the network's factors guarded
    by the HOSVD start."""
    Gtr, _ = pipeline_cores(P, 0, 8192)
    Gev, Uev = pipeline_cores(P, 100000, 512)
    net = P.MLP((R, R, R), R, (1024, 1024))
    W, b = synth.mlp_weights(77, net.dims)
    W[2] = W[2] * 0.1
    net.load(W, b)
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    losses = []
    epochs = 24
    for ep in range(epochs):
        perm = torch.randperm(Gtr.shape[0], device="cuda", generator=gen)
        lr = 1e-3 * 0.5 ** (ep // 6)
        ls = [net.train_step(Gtr[perm[i:i + 256]].contiguous(), lr)
              for i in range(0, Gtr.shape[0], 256)]
        losses.append(float(torch.cat(ls).mean()))
    assert losses[-1] < 0.1 * losses[0]          # the network learned the cores
    del Gtr
    Vs = net.split(net.forward(Gev))
    rng = np.random.default_rng(5512)
    its = {"random": [], "hosvd": [], "learned": []}
    fits = {k: [] for k in its}
    ms = {k: 0.0 for k in its}
    stream = torch.cuda.current_stream()
    for k in range(Gev.shape[0]):
        G = Gev[k].contiguous()
        starts = {
            "random": dict(init="user", A_init=[torch.from_numpy(synth.f32(
                rng.standard_normal((I, R)))).cuda() for _ in range(3)]),
            "hosvd": dict(init="hosvd"),
            "learned": dict(init="coeff_guarded", A_init=[v[k].contiguous() for v in Vs]),
        }
        for arm, kw in starts.items():
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            f = P.ffcp(Uev[k], G, R, update="als", max_it=1000, tol=1e-6, **kw)
            e1.record(stream)
            e1.synchronize()
            ms[arm] += e0.elapsed_time(e1)
            its[arm].append(int(f["info"]["iterations"]))
            fits[arm].append(float(f["info"]["fit"]))
    it = {k: np.array(v) for k, v in its.items()}
    print("held-out cores: 512; mean ALS iterations " +
          ", ".join(f"{k} {it[k].mean():.1f}" for k in it) +
          "; total FFCP ms " + ", ".join(f"{k} {ms[k]:.1f}" for k in ms), flush=True)
    # measured: random 243.5, HOSVD 352.1, learned 252.4 mean iterations.  On
    # cores of highly congruent CP models the HOSVD start (orthogonal
    # directions of the core) lands far from the solution; the network's
    # start removes that cost and ends level with a random start, whose
    # iterations are spent in the same slow final phase
    assert it["learned"].mean() < 0.8 * it["hosvd"].mean()
    assert it["learned"].mean() < 1.1 * it["random"].mean()
    # the guard keeps the start with the better initial fit; from a
    # different start ALS may end in a different local optimum, so the final
    # fits are compared over the set: the median difference is not negative
    # (measured: mean -1.0e-4, carried by one core at -3.9e-2), and the
    # learned arm ends worse by more than 1e-3 on at most 5 % of the cores
    # (measured 0.6 %)
    fl, fh = np.array(fits["learned"]), np.array(fits["hosvd"])
    worse = float(np.mean(fl < fh - 1e-3))
    print(f"final fit: learned - HOSVD mean {np.mean(fl - fh):.2e}, "
          f"min {np.min(fl - fh):.2e}; worse by > 1e-3 on {100 * worse:.1f} % of cores",
          flush=True)
    assert np.median(fl - fh) >= -1e-6
    assert worse <= 0.05
