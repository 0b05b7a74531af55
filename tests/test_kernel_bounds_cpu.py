"""CPU bounds check of every HIP kernel of the library.

The kernels (fwi_kernels.hip, deblur_kernels.hip) and the host code that
plans and launches them (fwi_api.hip, deblur_api.hip) are compiled for the
CPU against a stand-in HIP header (tests/kernel_emu): every GPU thread runs
as a fiber, blocks run one after another with their barriers and wavefront
shuffles, and every device buffer is an exact-size host allocation, so
AddressSanitizer aborts on any kernel access outside a buffer. The raw
buffer loads/stores of the step kernels are emulated from their descriptor
(base, range) and offsets.

The driver calls every public entry point through the C ABI on small
geometries built to reach the edge cases of the wave tables - ragged windows
and record lengths, strips and row bands without receivers (including the
last waves of the table), receivers just outside a row band - for every
tiling the autotuner can choose, with and without checkpointing, and the
autotuner itself; and the deblurring network on a grid with odd coarse
levels and on a width that selects the 128 x 128 GEMM and weight-gradient
kernels, split K and the direct input-layer kernels.
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

from synth import configs  # noqa: E402
from synth.problem import Acquisition, Grid  # noqa: E402
from synth.wavelet import ricker  # noqa: E402

EMU = os.path.join(ROOT, "tests", "kernel_emu")
CSRC = os.path.join(ROOT, "paper_2403_17518_amd", "csrc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SOURCES = ["fwi_kernels", "fwi_api", "deblur_kernels", "deblur_api"]
HEADERS = ["internal.h", "deblur_internal.h"]
# the autotuner's candidates (cw, rows, levels, prefetch) and checkpointed runs
TILINGS = [
    "1,8,1,1,0", "1,16,1,1,0", "1,24,1,1,0", "1,32,1,1,0", "1,48,1,1,0", "2,8,1,1,0", "2,16,1,1,0",
    "2,24,1,1,0", "2,32,1,1,0", "1,8,1,2,0", "1,16,1,2,0", "1,24,1,2,0", "1,32,1,2,0", "1,48,1,2,0",
    "2,8,1,2,0", "2,16,1,2,0", "2,24,1,2,0", "2,32,1,2,0", "1,24,2,1,0", "1,48,2,1,0", "2,24,2,1,0",
    "2,48,2,1,0", "1,24,2,2,0", "1,48,2,2,0", "1,96,2,2,0", "2,24,2,2,0", "2,48,2,2,0", "2,96,2,2,0",
    "1,16,2,1,0", "1,16,2,2,0", "2,16,2,2,0", "1,32,2,2,0", "2,32,2,2,0",
    "1,24,1,1,3", "2,16,1,2,3", "1,24,2,1,3", "2,48,2,1,2", "2,24,2,2,3", "auto",
    # binomial checkpointing: a snapshot cap below the uniform schedule's
    "1,24,1,1,1,1", "2,16,1,2,2,0", "1,24,2,1,1,2",
]

pytestmark = pytest.mark.skipif(not os.path.exists(CLANG), reason="ROCm clang++ not found")


def _patch(src: str) -> str:
    # bind the raw-buffer intrinsics to the emulation, route dynamic LDS
    # through the runtime and read the constant address space as ordinary
    # memory (which the address sanitizer checks); nothing else in the
    # sources changes
    for kind in ("load.f32", "load.v2f32", "load.v4f32", "store.f32", "store.v2f32"):
        name = "emu_raw_" + ("st_" if kind.startswith("store") else "ld_") + kind.split(".")[1]
        src = src.replace(f"llvm.amdgcn.raw.buffer.{kind}\")", f"{name}\")")
    src = src.replace("__attribute__((address_space(4)))", "")
    return re.sub(r"extern __shared__ float (\w+)\[\];", r"float *\1 = static_cast<float *>(emu_dyn_shared());", src)


@pytest.fixture(scope="module")
def emu_driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("kernel_emu")
    os.makedirs(d / "pkg" / "csrc")
    os.makedirs(d / "include")
    for h in ("fwi.h", "deblur.h"):
        shutil.copy(os.path.join(ROOT, "include", h), d / "include" / h)
    for name in [s + ".hip" for s in SOURCES] + HEADERS:
        with open(os.path.join(CSRC, name)) as f:
            text = _patch(f.read())
        with open(d / "pkg" / "csrc" / name, "w") as f:
            f.write(text)
    flags = ["-std=c++17", "-O2", "-g", "-w", "-fno-omit-frame-pointer", "-fsanitize=address",
             "-I", EMU, "-I", str(d / "include")]
    jobs, objs = [], []
    units = [(str(d / "pkg" / "csrc" / f"{s}.hip"), True) for s in SOURCES]
    units += [(os.path.join(EMU, "emu_rt.cpp"), False), (os.path.join(EMU, "emu_driver.cpp"), False)]
    for path, is_hip in units:
        obj = str(d / (os.path.basename(path) + ".o"))
        cmd = [CLANG, *flags, *(["-x", "c++"] if is_hip else []), "-c", path, "-o", obj]
        jobs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT))
        objs.append(obj)
    for p in jobs:
        out = p.communicate()[0]
        assert p.returncode == 0, out.decode()[-4000:]
    exe = str(d / "emu_driver")
    subprocess.run([CLANG, "-fsanitize=address", *objs, "-o", exe], check=True)
    return exe


ASAN_ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:detect_stack_use_after_return=0:abort_on_error=0")


def _run(exe, args, timeout):
    p = subprocess.run([exe, *args], capture_output=True, text=True, timeout=timeout, env=ASAN_ENV)
    assert p.returncode == 0, (p.stdout[-2000:] + "\n" + p.stderr[-6000:])
    return p.stdout


def _run_parallel(exe, fixed, items, nproc=4, timeout=900):
    """Runs exe fixed + chunk for `nproc` chunks of `items` at once."""
    chunks = [items[i::nproc] for i in range(nproc)]
    procs = [subprocess.Popen([exe, *fixed, *c], stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True,
                              env=ASAN_ENV) for c in chunks if c]
    outs = []
    for p in procs:
        out, err = p.communicate(timeout=timeout)
        assert p.returncode == 0, (out[-2000:] + "\n" + err[-6000:])
        outs.append(out)
    return "".join(outs)


def _write_geom(path, grid, acq, v0, vt):
    S = int(acq.nshots)
    has_win, has_nt = acq.win_x0 is not None, acq.nt is not None
    wav = np.asarray(acq.wavelet)
    frac = acq.src_fz is not None
    lines = [f"{grid.nz} {grid.nx} {grid.nb} {grid.h} {grid.dt} {grid.nt_max} {grid.v_ref} {grid.R} "
             f"{S} {int(has_win)} {int(has_nt)} {int(wav.ndim == 1)} {int(frac)} {int(grid.free_surface)} "
             f"{int(grid.pml)}"]
    for s in range(S):
        r0, r1 = int(acq.rec_ptr[s]), int(acq.rec_ptr[s + 1])
        x0 = int(acq.win_x0[s]) if has_win else 0
        wn = int(acq.win_nx[s]) if has_win else grid.nx
        nt = int(acq.nt[s]) if has_nt else grid.nt_max
        sf = (float(acq.src_fz[s]), float(acq.src_fx[s])) if frac else (0.0, 0.0)
        lines.append(f"{int(acq.src_z[s])} {int(acq.src_x[s])} {x0} {wn} {nt} {r1 - r0} {sf[0]!r} {sf[1]!r}")
        lines.append(" ".join(
            f"{int(acq.rec_z[r])} {int(acq.rec_x[r])} "
            f"{float(acq.rec_fz[r]) if frac else 0.0!r} {float(acq.rec_fx[r]) if frac else 0.0!r}"
            for r in range(r0, r1)))
    lines.append(" ".join(f"{float(w):.6e}" for w in wav[..., :grid.nt_max].ravel()))
    lines.append(" ".join(f"{float(v):.3f}" for v in np.asarray(v0, np.float32).ravel()))
    lines.append(" ".join(f"{float(v):.3f}" for v in np.asarray(vt, np.float32).ravel()))
    with open(path, "w") as f:
        f.write("\n".join(lines) + "\n")


def edge_geometry(nt_max: int = 8):
    """Three shots: a full-width window whose receivers cover only its left
    quarter and whose record is the shortest (so it takes the last slot: its
    top-band strips without receivers end the wave table), a narrow odd
    window, and a window with receivers 16 rows down (next to a row-band
    boundary) and a co-located pair."""
    grid = Grid(nz=30, nx=260, nb=10, h=10.0, dt=1e-3, nt_max=nt_max, v_ref=2400.0)
    rec = [[(2, x) for x in range(0, 60)],
           [(2, x) for x in range(100, 137)],
           [(16, x) for x in range(140, 150)] + [(16, 145)]]
    ptr = np.zeros(4, np.int64)
    for s in range(3):
        ptr[s + 1] = ptr[s] + len(rec[s])
    allr = [r for shot in rec for r in shot]
    acq = Acquisition(src_z=np.array([2, 2, 2], np.int32), src_x=np.array([30, 118, 200], np.int32),
                      rec_ptr=ptr, rec_z=np.array([r[0] for r in allr], np.int32),
                      rec_x=np.array([r[1] for r in allr], np.int32),
                      wavelet=ricker(20.0, grid.dt, nt_max),
                      win_x0=np.array([0, 100, 140], np.int32), win_nx=np.array([260, 37, 120], np.int32),
                      nt=np.array([nt_max - 3, nt_max, nt_max - 1], np.int32))
    z = np.arange(grid.nz, dtype=np.float32)[:, None]
    vt = np.broadcast_to(2000.0 + 10.0 * z, (grid.nz, grid.nx)).copy()
    vt[12:18, 100:160] += 150.0
    v0 = np.broadcast_to(2000.0 + 10.0 * z, (grid.nz, grid.nx)).copy()
    return grid, acq, v0, vt


def offgrid_geometry(nt_max: int = 8):
    """The edge geometry with every source and most receivers between grid
    points (bilinear spreading), including the last column of a window and
    the last model row left on the grid where the next cell does not exist."""
    grid, acq, v0, vt = edge_geometry(nt_max)
    rng = np.random.default_rng(11)
    nr = acq.rec_z.shape[0]
    fz = rng.uniform(0.0, 1.0, nr).astype(np.float32)
    fx = rng.uniform(0.0, 1.0, nr).astype(np.float32)
    fz[::5] = 0.0
    fx[::7] = 0.0
    for s in range(acq.nshots):
        a, b = acq.rec_ptr[s], acq.rec_ptr[s + 1]
        last = acq.win_x0[s] + acq.win_nx[s] - 1
        fx[a:b][acq.rec_x[a:b] == last] = 0.0
    fz[acq.rec_z == grid.nz - 1] = 0.0
    acq.rec_fz, acq.rec_fx = fz, fx
    acq.src_fz = np.array([0.25, 0.5, 0.0], np.float32)
    acq.src_fx = np.array([0.75, 0.0, 0.5], np.float32)
    return grid, acq, v0, vt


def free_surface_geometry(nt_max: int = 8):
    """The off-grid edge geometry under a pressure-free top surface (no top
    sponge, odd mirror rows above the surface)."""
    from dataclasses import replace
    grid, acq, v0, vt = offgrid_geometry(nt_max)
    return replace(grid, free_surface=True), acq, v0, vt


def pml_geometry(nt_max: int = 8):
    """The off-grid edge geometry with a perfectly matched layer."""
    from dataclasses import replace
    grid, acq, v0, vt = offgrid_geometry(nt_max)
    return replace(grid, pml=True), acq, v0, vt


def pml_free_surface_geometry(nt_max: int = 8):
    """The layer on three sides under a pressure-free top surface."""
    from dataclasses import replace
    grid, acq, v0, vt = offgrid_geometry(nt_max)
    return replace(grid, pml=True, free_surface=True), acq, v0, vt


def _ragged(nt_max: int = 8):
    wl = configs.ragged_small()
    g = wl.grid
    grid = Grid(nz=g.nz, nx=g.nx, nb=g.nb, h=g.h, dt=g.dt, nt_max=nt_max, v_ref=g.v_ref, R=g.R)
    a = wl.acq
    nt = None if a.nt is None else np.maximum(1, np.asarray(a.nt) * nt_max // g.nt_max).astype(np.int32)
    acq = Acquisition(src_z=a.src_z, src_x=a.src_x, rec_ptr=a.rec_ptr, rec_z=a.rec_z, rec_x=a.rec_x,
                      wavelet=np.asarray(a.wavelet)[..., :nt_max], win_x0=a.win_x0, win_nx=a.win_nx, nt=nt)
    return grid, acq, wl.v0, wl.v_true


def test_edge_geometry_has_receiverless_last_waves():
    """The edge geometry really ends the slot order with the shot whose
    right-hand strips hold no receivers."""
    grid, acq, _, _ = edge_geometry()
    order = sorted(range(acq.nshots), key=lambda s: -int(acq.nt[s]))
    last = order[-1]
    assert int(acq.rec_x[acq.rec_ptr[last]:acq.rec_ptr[last + 1]].max()) < grid.nx // 4
    assert int(acq.win_nx[last]) == grid.nx


@pytest.mark.parametrize("geom", ["edge", "ragged", "offgrid", "free_surface", "pml", "pml_free_surface"])
def test_step_kernels_in_bounds_every_tiling(emu_driver, tmp_path, geom):
    grid, acq, v0, vt = {"edge": edge_geometry, "ragged": _ragged, "offgrid": offgrid_geometry,
                         "free_surface": free_surface_geometry, "pml": pml_geometry,
                         "pml_free_surface": pml_free_surface_geometry}[geom]()
    path = str(tmp_path / "geom.txt")
    _write_geom(path, grid, acq, v0, vt)
    # every tiling, two levels per launch included, with and without the
    # layer and the free surface
    specs = list(TILINGS)
    out = _run_parallel(emu_driver, ["fd", path], specs)
    assert out.count("ok ") == len(specs), out
    # every tiling computes each cell with the same arithmetic: one set of bits
    hashes = {l.split("hash=")[1] for l in out.splitlines() if l.startswith("ok ")}
    assert len(hashes) == 1, out


@pytest.mark.parametrize("pml", [False, True])
def test_checkpoint_schedules_give_the_same_bits(emu_driver, tmp_path, pml):
    """Gradients and migrated images are the same bits with the whole
    history stored, uniform checkpoints, and binomial schedules down to no
    snapshot at all (every segment recomputed from the zero state); with the
    layer the snapshots carry its edge fields."""
    from dataclasses import replace
    grid, acq, v0, vt = _ragged()
    grid = replace(grid, pml=pml)
    path = str(tmp_path / "geom.txt")
    _write_geom(path, grid, acq, v0, vt)
    groups = {"1,24,1,1": ["0", "3", "1", "1,0", "1,1", "1,3", "2,0"],
              "1,24,2,1": ["0", "3", "1,0", "1,2"]}
    specs = [f"{t},{c}" for t, cs in groups.items() for c in cs]
    out = _run_parallel(emu_driver, ["fd", path], specs)
    lines = [l for l in out.splitlines() if l.startswith("ok ")]
    assert len(lines) == len(specs), out
    info = {l.split()[1]: dict(kv.split("=") for kv in l.split()[2:]) for l in lines}
    for t, cs in groups.items():
        hashes = {info[f"{t},{c}"]["hash"] for c in cs}
        assert len(hashes) == 1, (t, {c: info[f"{t},{c}"] for c in cs})
    # and one level per launch gives the bits of two
    assert len({i["hash"] for i in info.values()}) == 1, info
    # the capped schedules really ran with fewer snapshots and recomputed more
    assert int(info["1,24,1,1,1,0"]["slots"]) == 0
    assert int(info["1,24,1,1,1,0"]["recomputed"]) > int(info["1,24,1,1,1"]["recomputed"])


# (depth, base width, grid) -> kernels the configuration must reach
NET_CASES = {
    # odd coarse levels (5 x 7); weight-gradient tiles of 32, 64 and 128 rows
    (3, 32, 40, 56): ("k_gemm_v<", "k_wgrad_t<32, 128,", "k_wgrad_t<64, 128,", "k_wgrad_t<128, 128,", "k_pool_fwd",
                      "k_conv1_fwd", "k_wgrad_finish"),
    (1, 128, 64, 240): ("k_gemm2", "k_gemm_finish", "k_wgrad_t<128, 128,", "k_conv1_wgrad"),  # wide level 0
    # deep, narrow: split K with the scatter epilogue; bias of the transposed
    # convolutions from the gathered gradient
    (2, 256, 16, 16): ("k_gemm_finish", "k_wgrad_finish"),
    # narrow transposed convolution (N = 4 x 8): 64 x 64 weight-gradient tiles
    (1, 8, 32, 48): ("k_wgrad_t<64, 64,",),
}


@pytest.mark.parametrize("case", list(NET_CASES))
def test_network_kernels_in_bounds(emu_driver, case):
    depth, base, H, W = case
    out = _run(emu_driver, ["net", str(depth), str(base), str(H), str(W), str(H - 4), str(W - 6)], timeout=900)
    assert "ok net" in out
    for k in NET_CASES[case]:
        assert k in out, (k, out)
