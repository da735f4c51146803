"""Learned CGLS warm start on the GPU.

Training data: seeded random-ellipsoid phantoms voxelised on the GPU,
projected by relaxed CVP (with elevation correction), Gaussian noise of
sigma = noise_frac * rms of the clean projections, then the first two CGLS
iterates from zero.  The U-Net maps the two iterates to a warm start x0 (a
residual on the second iterate).  The training target is either the phantom
or (default) the CGLS iterate after target_iters iterations from zero: with
noisy data CGLS converges to the least-squares solution, not to the phantom,
and a start near the phantom still leaves the noise to be fitted.
Evaluation runs CGLS to rho <= tol from zero and from the warm start, with
rho = |A^T (b - A x)| / |A^T b| (the same denominator for both); the warm
start's cost includes its two initial iterations and the network inference.
Plain CGLS from zero is the fallback and the judge of the residual.

Run as a module for the held-out experiment:
  python -m paper_2110_09841_amd.warmstart --train 2000 --eval 200
"""
import argparse
import ctypes
import json
import time

import numpy as np
import torch

from . import _lib, synth
from .cgls import CGLS, BatchedCGLS
from .cvp import Batch, Geometry, Options, project
from .unet import UNet

HELD_OUT_SEED0 = 100000


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


class Pipeline:
    def __init__(self, params=None, n_ellipsoids=16, noise_frac=0.01,
                 opts=Options(variant="relaxed", ec=True), per_graph=5, target="cgls", target_iters=20):
        self.params = params or synth.config_warmstart()
        self.geom = Geometry(self.params)
        self.opts = opts
        self.n_ellipsoids = n_ellipsoids
        self.noise_frac = noise_frac
        self.shape = self.geom.vol_shape
        self.b = torch.empty(self.geom.proj_shape, dtype=torch.float32, device="cuda")
        self.solver = CGLS(self.geom, opts, self.b)
        self.per_graph = per_graph
        self.solver.capture(per_graph)          # captured once, outside any timing
        if target not in ("cgls", "phantom"):
            raise ValueError("target must be 'cgls' or 'phantom'")
        self.target, self.target_iters = target, int(target_iters)
        self._dims = (ctypes.c_int32 * 3)(*self.params["vol_dims"])
        self._vox = (ctypes.c_double * 3)(*self.params["voxel_mm"])

    def phantom(self, seed):
        """Ellipsoid phantom of draw_ellipsoids(seed), voxelised on the GPU."""
        ells, _ = synth.draw_ellipsoids(self.params["vol_dims"], self.params["voxel_mm"], self.n_ellipsoids, seed)
        d = torch.from_numpy(ells).cuda()
        x = torch.empty(self.shape, dtype=torch.float32, device="cuda")
        _lib.check(_lib.lib().cvp_synth_ellipsoids(ctypes.c_void_p(d.data_ptr()), len(ells), self._dims, self._vox,
                                                   ctypes.c_void_p(x.data_ptr()), _stream()))
        return x

    def measure(self, x_true, seed, out=None):
        """b = A x_true + N(0, (noise_frac * rms(A x_true))^2)."""
        b = project(x_true, self.geom, self.opts, out=out)
        rms = float(torch.sqrt((b.double() ** 2).mean()))
        _lib.check(_lib.lib().cvp_synth_add_gaussian(ctypes.c_void_p(b.data_ptr()), b.numel(),
                                                     ctypes.c_float(self.noise_frac * rms),
                                                     ctypes.c_uint64(1000003 * seed + 17), _stream()))
        return b

    def iterates(self, b):
        """The first two CGLS iterates from zero (copies)."""
        self.solver.reset(b)
        self.solver.set_tolerance(0.0)
        self.solver.start()
        self.solver.iterate(1)
        x1 = self.solver.x.clone()
        self.solver.iterate(1)
        return x1, self.solver.x.clone()

    def sample(self, seed):
        """(x1, x2, target) for the phantom of this seed."""
        x_true = self.phantom(seed)
        b = self.measure(x_true, seed, out=self.b)
        x1, x2 = self.iterates(b)
        if self.target == "phantom":
            return x1, x2, x_true
        self.solver.iterate(self.target_iters - 2)
        return x1, x2, self.solver.x.clone()

    def dataset(self, seeds, log=None):
        out = []
        for n, s in enumerate(seeds):
            out.append(self.sample(s))
            if log and (n + 1) % 200 == 0:
                torch.cuda.synchronize()
                log("generated %d / %d" % (n + 1, len(seeds)))
        return out

    def train(self, net: UNet, data, epochs=2, lr=1e-3, seed=0, log=None):
        """Adam on the MSE to the phantom, one sample per step, shuffled each
        epoch.  Returns the mean sampled loss per epoch."""
        rng = np.random.default_rng(seed)
        losses = []
        for ep in range(epochs):
            sampled = []
            for n, i in enumerate(rng.permutation(len(data))):
                loss = net.train_step(*data[i], lr=lr)
                if n % 50 == 0:
                    sampled.append(float(loss))      # synchronises
            losses.append(float(np.mean(sampled)))
            if log:
                log("epoch %d: mean sampled loss %.4e" % (ep, losses[-1]))
        return losses

    def evaluate(self, net: UNet, seed, tol=1e-3, max_iter=400):
        """Iterations and seconds to rho <= tol from zero and from the warm
        start on the held-out phantom of this seed."""
        x_true = self.phantom(seed)
        b = self.measure(x_true, seed).clone()
        self.solver.reset(b)
        it0, t0, rho0 = self.solver.run(tol=tol, max_iter=max_iter, per_graph=self.per_graph)
        gamma_ref = float(self.solver.gamma_history()[0])        # |A^T b|^2
        err0 = float(torch.linalg.vector_norm(self.solver.x - x_true) / torch.linalg.vector_norm(x_true))
        torch.cuda.synchronize()
        ts = time.perf_counter()
        x1, x2 = self.iterates(b)
        x0 = net.forward(x1, x2)
        self.solver.reset(None, x0)
        itw, _, rhow = self.solver.run(tol=tol, max_iter=max_iter, per_graph=self.per_graph, gamma_ref=gamma_ref)
        t_warm = time.perf_counter() - ts
        errw = float(torch.linalg.vector_norm(self.solver.x - x_true) / torch.linalg.vector_norm(x_true))
        return dict(seed=seed, zero_iters=it0, zero_s=t0, warm_iters=itw + 2, warm_s=t_warm,
                    rho0_warm=float(rhow[0]), reached_zero=bool(rho0[it0] <= tol),
                    reached_warm=bool(rhow[itw] <= tol), err_zero=err0, err_warm=errw)


def evaluate_batched(pipe: Pipeline, net: UNet, seeds, tol=1e-3, max_iter=400, per_graph=5):
    """The held-out phantoms of `seeds` as one batch (one geometry per
    problem, the same trajectory): batched CGLS from zero to rho <= tol
    against the warm start -- two batched CGLS iterations, the network on
    each problem's iterates, then batched CGLS from x0 to the same rho (the
    denominator |A^T b| of the zero start).  Every problem stops on the
    device when it meets the tolerance.  Returns per-problem iterations and
    the two wall times (the warm one including its two iterations and the
    inference)."""
    n = len(seeds)
    geoms = [Geometry(pipe.params) for _ in range(n)]
    batch = Batch(geoms)
    xt = [pipe.phantom(s) for s in seeds]
    bs = [pipe.measure(x, s).clone() for x, s in zip(xt, seeds)]
    zero = BatchedCGLS(batch, pipe.opts, bs)
    its0, t0, rhos0 = zero.run(tol=tol, max_iter=max_iter, per_graph=per_graph)
    refs = [float(g[0]) for g in zero.gamma_histories()]
    err0 = [float(torch.linalg.vector_norm(zero.x[q] - xt[q]) / torch.linalg.vector_norm(xt[q])) for q in range(n)]
    warm = BatchedCGLS(batch, pipe.opts, bs)
    warm.capture(per_graph)
    torch.cuda.synchronize()
    ts = time.perf_counter()
    warm.set_tolerance(0.0)
    warm.start()
    warm.iterate(1)
    x1 = [x.clone() for x in warm.x]
    warm.iterate(1)
    for q in range(n):
        # forward returns the network's own output buffer: copy before the next call
        warm.x[q].copy_(net.forward(x1[q], warm.x[q]))
    itsw, _, rhosw = warm.run(tol=tol, max_iter=max_iter, per_graph=per_graph, gamma_refs=refs)
    t_warm = time.perf_counter() - ts
    errw = [float(torch.linalg.vector_norm(warm.x[q] - xt[q]) / torch.linalg.vector_norm(xt[q])) for q in range(n)]
    return dict(seeds=list(seeds), zero_iters=its0, warm_iters=[i + 2 for i in itsw], zero_s=t0, warm_s=t_warm,
                rho0_warm=[float(r[0]) for r in rhosw], reached_zero=[bool(r[i] <= tol) for r, i in zip(rhos0, its0)],
                reached_warm=[bool(r[i] <= tol) for r, i in zip(rhosw, itsw)], err_zero=err0, err_warm=errw)


def main():
    ap = argparse.ArgumentParser(description="learned CGLS warm start: train, then evaluate on held-out phantoms")
    ap.add_argument("--train", type=int, default=2000, help="training phantoms (seeds 0 .. n-1)")
    ap.add_argument("--eval", type=int, default=200, help="held-out phantoms (seeds 100000 ..)")
    ap.add_argument("--epochs", type=int, default=2)
    ap.add_argument("--target", default="cgls", choices=["cgls", "phantom"])
    ap.add_argument("--target-iters", type=int, default=20)
    ap.add_argument("--save", default=None, help="write the trained parameters here (torch.save of a dict)")
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--tol", type=float, default=1e-3)
    ap.add_argument("--max-iter", type=int, default=400)
    ap.add_argument("--out", default=None, help="write the JSON record here as well")
    ap.add_argument("--batch", type=int, default=8, help="held-out phantoms per batched evaluation")
    args = ap.parse_args()

    def log(msg):
        print(msg, flush=True)

    torch.cuda.set_device(0)
    pipe = Pipeline(target=args.target, target_iters=args.target_iters)
    net = UNet(pipe.shape, seed=1)
    t0 = time.perf_counter()
    data = pipe.dataset(range(args.train), log=log)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    losses = pipe.train(net, data, epochs=args.epochs, lr=args.lr, log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    del data
    torch.cuda.empty_cache()
    if args.save:
        torch.save(net.state(), args.save)
    rows = []
    for n in range(args.eval):
        rows.append(pipe.evaluate(net, HELD_OUT_SEED0 + n, tol=args.tol, max_iter=args.max_iter))
        if (n + 1) % 10 == 0:
            r = rows[-1]
            log("eval %d / %d: zero %d it %.3f s, warm %d it %.3f s" % (n + 1, args.eval, r["zero_iters"], r["zero_s"],
                                                                      r["warm_iters"], r["warm_s"]))

    def stat(key):
        v = np.array([r[key] for r in rows], dtype=np.float64)
        return {"mean": float(v.mean()), "median": float(np.median(v)), "min": float(v.min()), "max": float(v.max())}

    # the same held-out phantoms through batched CGLS, args.batch at a time
    batches = []
    for n0 in range(0, args.eval, args.batch):
        seeds = [HELD_OUT_SEED0 + n for n in range(n0, min(n0 + args.batch, args.eval))]
        batches.append(evaluate_batched(pipe, net, seeds, tol=args.tol, max_iter=args.max_iter))
        log("batched eval %d / %d: zero %.3f s, warm %.3f s" % (n0 + len(seeds), args.eval, batches[-1]["zero_s"],
                                                             batches[-1]["warm_s"]))
    bz = np.concatenate([b["zero_iters"] for b in batches])
    bw = np.concatenate([b["warm_iters"] for b in batches])
    batched_rec = {"batch": args.batch, "batches": len(batches),
                   "zero_s": float(sum(b["zero_s"] for b in batches)),
                   "warm_s": float(sum(b["warm_s"] for b in batches)),
                   "zero_iters_mean": float(bz.mean()), "warm_iters_mean": float(bw.mean()),
                   "warm_fewer_iters": int(np.sum(bw < bz)),
                   "reached_zero": int(sum(sum(b["reached_zero"]) for b in batches)),
                   "reached_warm": int(sum(sum(b["reached_warm"]) for b in batches)),
                   "warm_faster_batches": int(sum(b["warm_s"] < b["zero_s"] for b in batches))}

    rec = {"workload": "warmstart_128c_180v", "train_phantoms": args.train, "eval_phantoms": args.eval,
           "epochs": args.epochs, "lr": args.lr, "tol": args.tol, "per_graph": pipe.per_graph,
           "target": args.target, "target_iters": args.target_iters if args.target == "cgls" else None,
           "data_s": t_data, "train_s": t_train, "epoch_loss": losses,
           "zero_iters": stat("zero_iters"), "warm_iters": stat("warm_iters"),
           "zero_s": stat("zero_s"), "warm_s": stat("warm_s"),
           "err_zero": stat("err_zero"), "err_warm": stat("err_warm"), "rho0_warm": stat("rho0_warm"),
           "reached_zero": int(sum(r["reached_zero"] for r in rows)),
           "reached_warm": int(sum(r["reached_warm"] for r in rows)),
           "warm_faster": int(sum(r["warm_s"] < r["zero_s"] for r in rows)),
           "batched": batched_rec}
    line = json.dumps(rec)
    print(line, flush=True)
    if args.out:
        with open(args.out, "w") as f:
            f.write(line + "\n")


if __name__ == "__main__":
    main()
