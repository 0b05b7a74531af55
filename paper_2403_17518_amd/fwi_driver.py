"""Full-waveform-inversion driver: plain gradient descent versus the
network-preconditioned update of the paper (section 2.3, Fig. 1).

One iteration of the network method:
  1. g_phi = fwi_gradient(v, d_obs)        (gradient of the misfit; the
     paper's gradient is g = -g_phi, eq. 13 with d_o - d_s)
  2. dm1 = born_pair(v, g) = born_mig(v, born_demig(v, g))   (doubly
     migrated image, eq. 15; one joint Born sweep feeds the migration)
  3. train the network dm1 -> g, warm-started from the previous iteration
     (transfer learning), reset at every new frequency band
  4. p = deblur_apply(g); if p is not a descent direction (<p, g_phi> >= 0)
     the plain direction p = g is used instead (the gradient stays the
     fallback and the reference for the descent test)
  5. line search along p and v <- clip(v + alpha p)
The plain method skips steps 2-4 (p = g). Both use the same line search:
a trial step with max|alpha p| = step_frac * v_max (shrunk by 4 until it
lowers the misfit, at most 4 times), a second at twice that, and the
minimiser of the parabola through the three misfits.

The paper's comparators (section 3.1): "bb", steepest descent with the
Barzilai-Borwein step alpha_short = (dx . dg) / (dg . dg) from the last two
models and gradients, and "lbfgs", the two-loop L-BFGS direction (memory 5).
Each takes its own step (alpha_short, resp. 1) as the trial of the shared
backtracking and accepts it when it lowers the misfit; the first iteration
of a band, which has no pair yet, uses the plain line search. "net" with
net_iters set runs the hybrid schedule: the network direction for the first
net_iters iterations of each band, the plain gradient afterwards.
Model quality is reported as the relative model error and as the SSIM
(structural similarity, Gaussian window) against the true model.

Multi-scale: the bands low-pass the data with a zero-phase 4th-order
Butterworth filter (the same filter applied to the wavelet); for synthetic
inputs the band's observed data are modelled with the filtered wavelet,
which is the same thing for a linear, time-invariant forward map.

Cost is counted two ways: wave-equation solves in the paper's convention
(gradient 2, demigration 1, migration 1, each misfit 1) and the stencil
passes the library actually ran.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from dataclasses import replace, dataclass, field

import numpy as np
import torch
from scipy.signal import butter, sosfiltfilt

from . import ops
from .deblur import DeblurConfig, DeblurNet


@dataclass
class FwiOptions:
    method: str = "plain"                 # "plain" or "net"
    bands: tuple = (3.0, 8.0, 15.0)       # low-pass corner frequencies (Hz)
    iters_per_band: int = 20
    step_frac: float = 0.01               # trial step: max|dv| = step_frac * v_max
    v_min: float = 1400.0
    v_max: float | None = None            # default: grid.v_ref
    train_steps_first: int = 500          # Adam steps in a band's first iteration
    train_steps: int = 200                # ... and in the later ones (warm start)
    lr: float = 1e-3
    diverge_factor: float = 100.0         # training whose loss ends above this x its start is discarded
    net: DeblurConfig = field(default_factory=DeblurConfig)
    seed: int = 2403
    mute_rows: int = 0                    # zero the update in the top rows (both methods)
    max_backtrack: int = 4                # trial-step reductions by 4 in the line search
    target_error: float | None = None     # stop once the model error is at or below this
    net_iters: int | None = None          # hybrid: network direction only in the first k iterations
    lbfgs_memory: int = 5
    qn_max_frac: float = 0.05             # cap of a BB / L-BFGS trial step: max|dv| <= this * v_max


# (depth, widths of the first level, LeakyReLU slope): a small network, and
# the paper's (four pooling levels, 128 to 2048 channels, slope 0.2; its
# network subsection and appendix table)
NETWORKS = {"small": (3, 32, 0.0), "paper": (4, 128, 0.2)}


def lowpass(x: np.ndarray, dt: float, fmax: float, axis: int = -1) -> np.ndarray:
    """Zero-phase 4th-order Butterworth low-pass (forward-backward)."""
    sos = butter(4, fmax, btype="low", fs=1.0 / dt, output="sos")
    return sosfiltfilt(sos, x, axis=axis)


def band_acq(acq, grid, fmax):
    w = np.asarray(acq.wavelet, dtype=np.float64)
    wf = lowpass(w, grid.dt, fmax).astype(np.float32)
    return replace_acq(acq, wf)


def replace_acq(acq, wavelet):
    from copy import copy
    a = copy(acq)
    a.wavelet = wavelet
    return a


def _sync():
    torch.cuda.synchronize()


class FwiRun:
    def __init__(self, fctx: ops.FwiContext, grid, acq, v0: np.ndarray, opts: FwiOptions,
                 v_true: np.ndarray | None = None, log=print):
        self.fctx, self.grid, self.acq, self.opts, self.log = fctx, grid, acq, opts, log
        self.dev = fctx.device
        self.v = torch.from_numpy(np.ascontiguousarray(v0, dtype=np.float32)).to(self.dev)
        self.v_true = None if v_true is None else torch.from_numpy(
            np.ascontiguousarray(v_true, dtype=np.float32)).to(self.dev)
        self.e0 = None if v_true is None else float(torch.linalg.norm(self.v - self.v_true))
        self.v_max = opts.v_max if opts.v_max is not None else float(grid.v_ref)
        self.step_scale = 1.0     # trial step relative to step_frac * v_max
        self.solves = 0           # paper convention
        self.passes = 0.0         # stencil passes actually run (one field, all shots)
        self.t0 = None
        self.history = []
        self.net = None
        if opts.method == "net":
            self.net = DeblurNet(fctx, opts.net, seed=opts.seed)
        self.v_true_np = None if v_true is None else np.asarray(v_true, np.float64)
        self._reset_pairs()

    def _reset_pairs(self):
        """Quasi-Newton memory (BB, L-BFGS): cleared at every band."""
        self.prev_v = None
        self.prev_g = None
        self.pairs = []

    def model_ssim(self) -> float | None:
        if self.v_true_np is None:
            return None
        vt = self.v_true_np
        return ssim(self.v.double().cpu().numpy(), vt, float(vt.max() - vt.min()))

    def model_error(self) -> float | None:
        if self.v_true is None:
            return None
        return float(torch.linalg.norm(self.v - self.v_true)) / self.e0

    def _count(self, solves: int):
        """Account one library call: paper-convention solves and the stencil
        passes it ran (cell-updates / updates of one field pass)."""
        self.solves += solves
        st = self.fctx.stats()
        self.passes += st["cell_updates"] / max(self._updates_per_pass, 1.0)

    def _misfit(self, acq, v, d_obs):
        phi = self.fctx.fwi_misfit(self.grid, acq, v, d_obs)
        self._count(1)
        return phi

    def run(self, observe) -> list:
        """observe(acq_band) -> d_obs (device tensor) for that band."""
        o = self.opts
        self._updates_per_pass = _updates_per_pass(self.grid, self.acq)
        self.t0 = time.perf_counter()
        for bi, fmax in enumerate(o.bands):
            acq_b = band_acq(self.acq, self.grid, fmax)
            d_obs = observe(acq_b)
            if self.net is not None and bi > 0:
                self.net.reset(o.seed + bi)      # a new band starts from scratch
            self.step_scale = 1.0
            self._reset_pairs()
            for it in range(o.iters_per_band):
                rec = self.iteration(acq_b, d_obs, bi, it, fmax)
                self.history.append(rec)
                self.log(json.dumps(rec))
                e = rec["model_error"]
                if o.target_error is not None and e is not None and e <= o.target_error:
                    return self.history
        return self.history

    def iteration(self, acq, d_obs, band, it, fmax):
        o = self.opts
        t = {}
        _sync()
        ta = time.perf_counter()
        use_net = self.net is not None and (o.net_iters is None or it < o.net_iters)
        dm1 = None
        if use_net and not o.mute_rows:
            # gradient and J^T J g in one call (the pair reuses the gradient's
            # stored imaging history when it fits in memory)
            g_phi, phi, dm1 = self.fctx.gradient_pair(self.grid, acq, self.v, d_obs, scale=-1.0)
            self._count(4)
        else:
            g_phi, phi, _ = self.fctx.fwi_gradient(self.grid, acq, self.v, d_obs)
            self._count(2)
        _sync()
        t["gradient"] = time.perf_counter() - ta
        g = -g_phi                                   # the paper's gradient
        if o.mute_rows:
            g[:o.mute_rows] = 0
        p = g
        fallback = None
        train_loss = None
        net_dir = False          # p is the network's direction
        a_qn = None              # quasi-Newton trial step along p
        if o.method in ("bb", "lbfgs"):
            p, a_qn = self._qn_direction(g_phi)
        if use_net:
            ta = time.perf_counter()
            if dm1 is None:
                # the pair J^T J g (demigration + migration, 2 solves) in one joint sweep
                dm1 = self.fctx.born_pair(self.grid, acq, self.v, g.contiguous())
                self._count(2)
            _sync()
            t["pair"] = time.perf_counter() - ta
            ta = time.perf_counter()
            steps = o.train_steps_first if it == 0 else o.train_steps
            hist = self.net.deblur_train(dm1, g.contiguous(), steps, o.lr)
            train_loss = [float(hist[0]), float(hist[-1])]
            if not (np.isfinite(train_loss[1]) and train_loss[1] <= o.diverge_factor * train_loss[0]):
                # training diverged: redraw the weights and take the plain
                # direction this iteration
                self.net.reset(o.seed + 7919 * (band + 1) + it)
                fallback = "diverged"
            else:
                q = self.net.deblur_apply(g.contiguous())
                if o.mute_rows:
                    q[:o.mute_rows] = 0
                fallback = not (float(torch.sum(q * g_phi)) < 0.0 and bool(torch.isfinite(q).all()))
                if not fallback:
                    p = q
                    net_dir = True
            _sync()
            t["train_apply"] = time.perf_counter() - ta
        # line search along p (shared by all methods)
        ta = time.perf_counter()
        pmax = float(p.abs().max())
        if not pmax > 0:
            return self._record(band, it, fmax, phi, t, 0.0, fallback, train_loss)
        self.prev_v, self.prev_g = self.v.clone(), g_phi.clone()
        scale0 = self.step_scale
        alpha = self._search(acq, d_obs, phi, p, pmax, a_qn)
        if alpha == 0.0 and net_dir:
            # no decrease along the network's direction: the plain gradient
            # takes this iteration, from the step scale that held before
            self.step_scale = scale0
            p, pmax = g, float(g.abs().max())
            fallback = "no decrease"
            alpha = self._search(acq, d_obs, phi, p, pmax, None)
        self.v = self._clip(self.v + alpha * p)
        _sync()
        t["line_search"] = time.perf_counter() - ta
        return self._record(band, it, fmax, phi, t, alpha * pmax, fallback, train_loss)

    def _search(self, acq, d_obs, phi, p, pmax, a_qn):
        """Step length along p that lowers the misfit (0 if none is found)."""
        o = self.opts
        if a_qn is not None:
            # the quasi-Newton step, capped and backtracked; accepted as soon
            # as it lowers the misfit
            a0 = min(a_qn, o.qn_max_frac * self.v_max / pmax)
            f1 = self._misfit(acq, self._clip(self.v + a0 * p), d_obs)
            nb = 0
            while f1 >= phi and nb < o.max_backtrack:
                a0 *= 0.25
                nb += 1
                f1 = self._misfit(acq, self._clip(self.v + a0 * p), d_obs)
            return a0 if f1 < phi else 0.0
        # trial step, shrunk by 4 while it does not reduce the misfit
        # (at most `max_backtrack` times), then a second point at twice it
        a0 = self.step_scale * o.step_frac * self.v_max / pmax
        f1 = self._misfit(acq, self._clip(self.v + a0 * p), d_obs)
        nb = 0
        while f1 >= phi and nb < o.max_backtrack:
            a0 *= 0.25
            nb += 1
            f1 = self._misfit(acq, self._clip(self.v + a0 * p), d_obs)
        if f1 < phi:
            f2 = self._misfit(acq, self._clip(self.v + 2 * a0 * p), d_obs)
            alpha = parabola_step(phi, f1, f2, a0)
            if alpha == 0.0:
                alpha = a0
        else:
            alpha = 0.0
        # the next trial starts from the scale that worked
        self.step_scale = min(1.0, self.step_scale * (0.25 ** nb) * (2.0 if nb == 0 else 1.0))
        return alpha

    def _qn_direction(self, g_phi):
        """Search direction and trial step of the BB or L-BFGS iteration."""
        o = self.opts
        if self.prev_v is not None:
            s_ = (self.v - self.prev_v).double()
            y_ = (g_phi - self.prev_g).double()
            sy = float(torch.sum(s_ * y_))
            if sy > 1e-12 * float(torch.linalg.norm(s_)) * float(torch.linalg.norm(y_)):
                self.pairs.append((s_, y_))
                self.pairs = self.pairs[-(o.lbfgs_memory if o.method == "lbfgs" else 1):]
        if not self.pairs:
            return -g_phi, None            # no curvature pair yet: plain line search
        if o.method == "bb":
            a = bb_short(*self.pairs[-1])
            return -g_phi, a
        d = -lbfgs_two_loop(g_phi, self.pairs)
        return d.float().contiguous(), 1.0

    def _clip(self, v):
        return torch.clamp(v, self.opts.v_min, self.v_max).contiguous()

    def _record(self, band, it, fmax, phi, t, step, fallback, train_loss):
        return {"method": self.opts.method, "band": band, "fmax": fmax, "iter": it, "misfit": phi,
                "model_error": self.model_error(), "ssim": self.model_ssim(), "solves": self.solves,
                "stencil_passes": round(self.passes, 3), "wall_s": time.perf_counter() - self.t0,
                "phase_s": {k: round(v, 4) for k, v in t.items()}, "max_dv": step,
                "fallback": fallback, "train_loss": train_loss}


def _updates_per_pass(grid, acq) -> float:
    tot = 0.0
    for s in range(len(acq.src_z)):
        wnx = grid.nx if acq.win_nx is None else int(acq.win_nx[s])
        nt = grid.nt_max if acq.nt is None else int(acq.nt[s])
        tot += (grid.nz + 2 * grid.nb) * (wnx + 2 * grid.nb) * nt
    return tot


def net_grid(nz: int, nx: int, depth: int) -> tuple[int, int]:
    """Smallest network grid holding an nz x nx image with at least one cell
    of reflect padding on each side and sides divisible by 2^depth."""
    q = 1 << depth

    def one(n):
        return ((n + 2 + q - 1) // q) * q

    return one(nz), one(nx)


def parabola_step(phi0: float, f1: float, f2: float, a0: float) -> float:
    """Step length from misfits at 0, a0 and 2 a0: the parabola's minimiser
    (clamped to [0, 4 a0]) when it is convex, else the better trial point."""
    curv = phi0 - 2 * f1 + f2
    if curv > 0:
        alpha = a0 * (3 * phi0 - 4 * f1 + f2) / (2 * curv)
        return min(max(alpha, 0.0), 4 * a0)
    if min(f1, f2) >= phi0:
        return 0.0
    return 2 * a0 if f2 < f1 else a0


def bb_short(dx: torch.Tensor, dg: torch.Tensor) -> float | None:
    """Barzilai-Borwein step alpha_short = (dx . dg) / (dg . dg) (the short
    step of the two-point method, eq. 17); None when it is not positive."""
    num = float(torch.sum(dx.double() * dg.double()))
    den = float(torch.sum(dg.double() * dg.double()))
    if not (den > 0.0) or not (num > 0.0):
        return None
    return num / den


def lbfgs_two_loop(g: torch.Tensor, pairs: list) -> torch.Tensor:
    """H g for the L-BFGS inverse-Hessian approximation built from the
    (s, y) pairs, oldest first (Liu and Nocedal's two-loop recursion, with
    H0 = (s.y)/(y.y) I from the newest pair)."""
    q = g.double().clone()
    alphas = []
    for s_, y_ in reversed(pairs):
        rho = 1.0 / float(torch.sum(y_ * s_))
        a = rho * float(torch.sum(s_ * q))
        alphas.append((a, rho))
        q -= a * y_
    s_, y_ = pairs[-1]
    q *= float(torch.sum(s_ * y_)) / float(torch.sum(y_ * y_))
    for (s_, y_), (a, rho) in zip(pairs, reversed(alphas)):
        b = rho * float(torch.sum(y_ * q))
        q += (a - b) * s_
    return q


def ssim(x: np.ndarray, y: np.ndarray, data_range: float, sigma: float = 1.5) -> float:
    """Mean structural similarity of two images (Wang et al. 2004): local
    means, variances and covariance under a Gaussian window (sigma 1.5,
    truncated at 3.5 sigma), K1 = 0.01, K2 = 0.03."""
    from scipy.ndimage import gaussian_filter
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    c1, c2 = (0.01 * data_range) ** 2, (0.03 * data_range) ** 2
    f = lambda a: gaussian_filter(a, sigma, mode="reflect", truncate=3.5)
    mx, my = f(x), f(y)
    vx = f(x * x) - mx * mx
    vy = f(y * y) - my * my
    cxy = f(x * y) - mx * my
    m = ((2 * mx * my + c1) * (2 * cxy + c2)) / ((mx * mx + my * my + c1) * (vx + vy + c2))
    return float(m.mean())


def time_to_error(plain: list, net: list) -> dict:
    """Iterations, solves and wall time the network method needs to reach
    the plain method's final model error."""
    target = plain[-1]["model_error"]
    out = {"target_model_error": target, "plain_iters": len(plain),
           "plain_wall_s": plain[-1]["wall_s"], "plain_solves": plain[-1]["solves"],
           "net_final_model_error": net[-1]["model_error"]}
    for k, r in enumerate(net):
        if r["model_error"] is not None and target is not None and r["model_error"] <= target:
            out.update({"net_iters": k + 1, "net_wall_s": r["wall_s"], "net_solves": r["solves"]})
            break
    else:
        out.update({"net_iters": None, "net_wall_s": None, "net_solves": None})
    return out


def rtm_scores(fctx, grid, acq, wl, fmax, finals, observe) -> dict:
    """Image score (normalised cross-correlation with the image migrated in
    the true model) of the RTM image of each final model and of the initial
    model, from the highest band's observed data with the direct arrival
    muted; the top 10 rows (source/receiver footprint) are left out."""
    from .rtm import image_score, rtm_image
    acq_b = band_acq(acq, grid, fmax)
    d_obs = observe(acq_b)
    w = np.abs(np.asarray(acq_b.wavelet, np.float64))
    t_peak = float(np.argmax(w)) * grid.dt
    mute = (float(np.min(wl.v0[0])), t_peak + 1.0 / fmax, 0.5 / fmax)
    dev = d_obs.device
    ref = rtm_image(fctx, grid, acq_b, torch.from_numpy(wl.v_true.astype(np.float32)).to(dev), d_obs, *mute)
    models = {"initial": torch.from_numpy(wl.v0.astype(np.float32)).to(dev), **finals}
    return {name: round(image_score(rtm_image(fctx, grid, acq_b, v, d_obs, *mute), ref, top=10), 4)
            for name, v in models.items()}


def main(argv=None):
    ap = argparse.ArgumentParser(description="plain vs network-preconditioned FWI on a seeded workload")
    ap.add_argument("--workload", default="salt_848x176")
    ap.add_argument("--method", default="both", choices=["plain", "net", "bb", "lbfgs", "both", "all"],
                    help="both = plain then net; all = plain, bb, lbfgs, net")
    ap.add_argument("--net-iters", type=int, default=0,
                    help="hybrid schedule: network direction only in a band's first k iterations")
    ap.add_argument("--iters", type=int, default=20, help="iterations per band")
    ap.add_argument("--bands", default="3,8,15")
    ap.add_argument("--shots", type=int, default=0)
    ap.add_argument("--net", default="small", choices=["small", "paper"],
                    help="small: depth 3, widths 32-256, ReLU; paper: the paper's network (Appendix A, "
                         "Table 1): depth 4, widths 128-2048, LeakyReLU 0.2")
    ap.add_argument("--lr", type=float, default=None,
                    help="peak learning rate of the network's Adam steps (default 1e-3 for the small "
                         "network, 1e-4 for the paper's)")
    ap.add_argument("--train-first", type=int, default=500)
    ap.add_argument("--train", type=int, default=200)
    ap.add_argument("--out", default="")
    ap.add_argument("--seed", type=int, default=None, help="network initialisation seed (default: the options' seed)")
    ap.add_argument("--rtm", action="store_true",
                    help="after the runs, score the RTM image of each final model (and of the initial model) "
                         "against the image migrated with the true model")
    ap.add_argument("--plain-log", default="",
                    help="log of an earlier plain run (JSON lines): the net run stops at its final "
                         "model error and the time-to-error summary is computed against it")
    args = ap.parse_args(argv)
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    from synth import configs
    wl = {"salt_848x176": lambda: configs.salt_848x176(args.shots or 100),
          "salt_1700x350": lambda: configs.salt_1700x350(args.shots or 300),
          "layered_600x200": lambda: configs.layered_600x200(args.shots or 64),
          "marmousi_601x221": lambda: configs.marmousi_601x221()}[args.workload]()
    grid, acq = wl.grid, wl.acq
    fctx = ops.FwiContext(0)
    v_true_t = torch.from_numpy(wl.v_true.astype(np.float32)).cuda()

    def observe(acq_b):
        return fctx.fwi_forward(grid, acq_b, v_true_t)

    depth, base, slope = NETWORKS[args.net]
    H, W = net_grid(grid.nz, grid.nx, depth)
    net_cfg = DeblurConfig(depth, base, slope, H, W)
    bands = tuple(float(b) for b in args.bands.split(","))
    out = {}
    lines = []

    def log(s):
        print(s, flush=True)
        lines.append(s)

    if args.plain_log:
        with open(args.plain_log) as f:
            out["plain"] = [r for r in (json.loads(x) for x in f if x.startswith("{"))
                            if r.get("method") == "plain"]
    methods = {"both": ["plain", "net"], "all": ["plain", "bb", "lbfgs", "net"]}.get(args.method, [args.method])
    finals = {}
    for method in methods:
        target = out["plain"][-1]["model_error"] if method == "net" and "plain" in out else None
        if args.method == "all":
            target = None          # full curves for the comparison
        lr = args.lr if args.lr is not None else (1e-3 if args.net == "small" else 1e-4)
        opts = FwiOptions(method=method, bands=bands, iters_per_band=args.iters, net=net_cfg,
                          train_steps_first=args.train_first, train_steps=args.train, lr=lr,
                          target_error=target, net_iters=args.net_iters or None)
        if args.seed is not None:
            opts = replace(opts, seed=args.seed)
        run = FwiRun(fctx, grid, acq, wl.v0, opts, v_true=wl.v_true, log=log)
        out[method] = run.run(observe)
        finals[method] = run.v.clone()
        if run.net is not None:
            run.net.close()
    if "plain" in out and "net" in out:
        summary = time_to_error(out["plain"], out["net"])
        summary["workload"] = wl.name
        log(json.dumps({"summary": summary}))
    if args.rtm:
        log(json.dumps({"rtm": rtm_scores(fctx, grid, acq, wl, bands[-1], finals, observe)}))
    if args.out:
        with open(args.out, "w") as f:
            f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
