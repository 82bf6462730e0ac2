"""Build liblupp.so (HIP, gfx950) in-tree.

    python -m paper_2609_15217_amd.build [-j JOBS]

Every kernel instance (one per size n for the thread path, one per (n, T) for
the lanes path) gets its own generated translation unit so that the
fully-unrolled kernels compile in parallel; a generated registry maps (n, T)
to the launchers. The list of compiled variants lives here.
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import json
import os
import re
import shutil
import subprocess
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
INCLUDE = os.path.join(ROOT, "include")
BUILD = os.path.join(ROOT, "_build", "lupp")
LIB = os.path.join(PKG, "liblupp.so")

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CXXFLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument", "-I", INCLUDE, "-I", CSRC,
]

THREAD_NS = list(range(1, 14))  # registers-only thread path


def lanes_widths(n: int) -> list[int]:
    """Segment widths T compiled for size n (K = ceil(n/T) rows per lane)."""
    if n == 2:
        return [2]
    if n <= 4:
        return [2, 4]
    if n <= 8:
        return [4, 8]
    if n <= 16:
        return [8, 16]  # T = 4 needs K >= 3 rows per lane here and spills
    return [16, 32]


LANES = [(n, t) for n in range(2, 33) for t in lanes_widths(n)]


def _write_if_changed(path: str, text: str):
    if os.path.exists(path) and open(path).read() == text:
        return
    with open(path, "w") as f:
        f.write(text)


def generate(gen: str) -> list[str]:
    os.makedirs(gen, exist_ok=True)
    srcs = []
    for n in THREAD_NS:
        p = os.path.join(gen, f"thread_{n}.hip")
        _write_if_changed(p, f'#include "kernels_thread.h"\nLUPP_THREAD_INSTANCE({n})\n')
        srcs.append(p)
    for n, t in LANES:
        p = os.path.join(gen, f"lanes_{n}_{t}.hip")
        _write_if_changed(p, f'#include "kernels_lanes.h"\n#include "kernels_lanes_soa.h"\nLUPP_LANES_INSTANCE({n}, {t})\n')
        srcs.append(p)
    for g in range(4):
        ns = [n for n in range(1, 33) if (n - 1) % 4 == g]
        p = os.path.join(gen, f"ragged_one_{g}.hip")
        _write_if_changed(p, '#include "kernels_ragged.h"\n' +
                          "".join(f"LUPP_RAGGED_ONE_INSTANCE({n})\n" for n in ns))
        srcs.append(p)
    # registry
    lines = ['#include "internal.h"', '#include "kernels_ragged.h"', "namespace lupp {"]
    for n in range(1, 33):
        lines.append(f"hipError_t ragged_one_launch_{n}(const RaggedArgs &, int, hipStream_t);")
    lines.append("hipError_t ragged_one_launch(int n, const RaggedArgs &a, int items, hipStream_t st) {\n  switch (n) {")
    lines += [f"  case {n}: return ragged_one_launch_{n}(a, items, st);" for n in range(1, 33)]
    lines.append("  default: return hipErrorInvalidValue;\n  }\n}")
    for n in THREAD_NS:
        lines.append(f"LaunchFn thread_fn_{n}(); const void *thread_sym_{n}();")
    for n, t in LANES:
        lines.append(f"LaunchFn lanes_fn_{n}_{t}(); const void *lanes_sym_{n}_{t}(int layout);")
    lines.append("LaunchFn thread_launcher(int n) {\n  switch (n) {")
    lines += [f"  case {n}: return thread_fn_{n}();" for n in THREAD_NS]
    lines.append("  default: return nullptr;\n  }\n}")
    lines.append("const void *thread_kernel_symbol(int n) {\n  switch (n) {")
    lines += [f"  case {n}: return thread_sym_{n}();" for n in THREAD_NS]
    lines.append("  default: return nullptr;\n  }\n}")
    lines.append("LaunchFn lanes_launcher(int n, int t) {")
    lines += [f"  if (n == {n} && t == {t}) return lanes_fn_{n}_{t}();" for n, t in LANES]
    lines.append("  return nullptr;\n}")
    lines.append("const void *lanes_kernel_symbol(int n, int t, int layout) {")
    lines += [f"  if (n == {n} && t == {t}) return lanes_sym_{n}_{t}(layout);" for n, t in LANES]
    lines.append("  return nullptr;\n}")
    lines.append("int lanes_widths(int n, int *out, int cap) {\n  int c = 0;")
    for n in range(2, 33):
        ws = lanes_widths(n)
        body = " ".join(f"if (c < cap) out[c] = {w}; ++c;" for w in ws)
        lines.append(f"  if (n == {n}) {{ {body} }}")
    lines.append("  return c;\n}")
    # autotuned defaults measured on gfx950
    tuned = {}
    tp = os.path.join(PKG, "dispatch_gfx950.json")
    if os.path.exists(tp):
        for e in json.load(open(tp)).get("entries", []):
            tuned[(int(e["n"]), 0 if e["layout"] == "aos" else 1, int(e["bucket"]))] = e
    lines.append("bool tuned_choice(int n, int layout, int bucket, int *v, int *l, int *w) {")
    for (n, lay, bk), e in sorted(tuned.items()):
        v = 1 if e["variant"] == "thread" else 2
        if v == 1 and n not in THREAD_NS:
            continue
        if v == 2 and (n, int(e["lanes"])) not in LANES:
            continue
        lines.append(f"  if (n == {n} && layout == {lay} && bucket == {bk}) {{ *v = {v}; *l = {int(e['lanes'])}; "
                     f"*w = {int(e['wpb'])}; return true; }}")
    lines.append("  (void)n; (void)layout; (void)bucket; (void)v; (void)l; (void)w;\n  return false;\n}")
    # lanes per size of the ragged path, measured by lupp_autotune_ragged
    ragged = {}
    if os.path.exists(tp):
        for e in json.load(open(tp)).get("ragged", []):
            ragged[int(e["n"])] = int(e["lanes"])
    lines.append("bool tuned_ragged(int n, int *lanes) {")
    for n, t in sorted(ragged.items()):
        lines.append(f"  if (n == {n}) {{ *lanes = {t}; return true; }}")
    lines.append("  (void)n; (void)lanes;\n  return false;\n}")
    lines.append("}  // namespace lupp")
    p = os.path.join(gen, "registry.hip")
    _write_if_changed(p, "\n".join(lines) + "\n")
    srcs.append(p)
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".cpp")):
            srcs.append(os.path.join(CSRC, name))
    return srcs


_INCLUDE_RE = re.compile(r'^\s*#\s*include\s*"([^"]+)"', re.M)


def _local_headers(src: str) -> list[str]:
    """Headers of this project that `src` includes, directly or not."""
    seen: dict[str, None] = {}
    todo = [src]
    while todo:
        f = todo.pop()
        for name in _INCLUDE_RE.findall(open(f, encoding="utf-8", errors="replace").read()):
            for d in (os.path.dirname(f), CSRC, INCLUDE):
                p = os.path.join(d, name)
                if os.path.exists(p):
                    p = os.path.realpath(p)
                    if p not in seen:
                        seen[p] = None
                        todo.append(p)
                    break
    return sorted(seen)


def _deps_hash(src: str) -> str:
    h = hashlib.sha256()
    h.update(" ".join(CXXFLAGS).encode())
    h.update(open(src, "rb").read())
    for p in _local_headers(src):
        h.update(p.encode())
        h.update(open(p, "rb").read())
    return h.hexdigest()[:20]


def _compile(src: str, obj_dir: str, force: bool) -> tuple[str, float, bool]:
    base = os.path.splitext(os.path.basename(src))[0]
    obj = os.path.join(obj_dir, base + ".o")
    stamp = obj + ".hash"
    hsh = _deps_hash(src)
    if not force and os.path.exists(obj) and os.path.exists(stamp) and open(stamp).read() == hsh:
        return obj, 0.0, False
    t0 = time.time()
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [HIPCC, *CXXFLAGS, *lang, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {src}\n{r.stderr[-4000:]}")
    with open(stamp, "w") as f:
        f.write(hsh)
    return obj, time.time() - t0, True


def build(jobs: int | None = None, force: bool = False, verbose: bool = True) -> str:
    """Compile every HIP translation unit (incrementally) and link liblupp.so."""
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        raise RuntimeError("hipcc not found")
    gen = os.path.join(BUILD, "gen")
    objd = os.path.join(BUILD, "obj")
    os.makedirs(objd, exist_ok=True)
    srcs = generate(gen)
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    t0 = time.time()
    objs, rebuilt = [], 0
    # largest kernels first so the pool stays busy
    order = sorted(srcs, key=lambda s: -_weight(s))
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = {ex.submit(_compile, s, objd, force): s for s in order}
        for f in cf.as_completed(futs):
            obj, dt, did = f.result()
            objs.append(obj)
            rebuilt += did
            if verbose and did:
                print(f"  [{rebuilt}] {os.path.basename(obj)} {dt:.1f}s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *sorted(objs)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    if verbose:
        print(f"liblupp.so: {len(objs)} objects ({rebuilt} rebuilt) in {time.time() - t0:.1f}s",
              flush=True)
    return LIB


def _weight(src: str) -> int:
    b = os.path.basename(src)
    if b.startswith("lanes_"):
        n, t = (int(v) for v in b[6:-4].split("_"))
        return n * n * ((n + t - 1) // t)
    if b.startswith("thread_"):
        n = int(b[7:-4])
        return 4 * n ** 3
    if b.startswith(("ragged_c", "grouped_c")):
        return 400_000
    if b.startswith("ragged"):
        return 200_000
    return 50_000 if "constitutive" in b else 0


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", "--jobs", type=int, default=None)
    ap.add_argument("--force", action="store_true")
    a = ap.parse_args()
    build(a.jobs, a.force)
    sys.exit(0)
