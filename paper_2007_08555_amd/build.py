"""Builds libmtp.so for gfx950 in-tree.

    python -m paper_2007_08555_amd.build [--jobs N] [--levels 8,16]

Steps: generate one evaluation kernel per compiled basis level
(codegen.py), compile every .hip source with hipcc for gfx950, link
paper_2007_08555_amd/libmtp.so.  Object files go to
paper_2007_08555_amd/_build/ and are reused while their source (for a part of
a generated kernel file: the sections that part compiles), the project
headers it includes and the flags are unchanged.  MTP_EXTRA_LEVELS (e.g.
"18") adds basis levels to the default ones (2-16 straight-line, 20 and 24
table-driven).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import hashlib
import re
import os
import shutil
import subprocess
import sys
import time

from . import codegen

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
GEN = os.path.join(CSRC, "generated")
BUILD = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmtp.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # keep the compiler from forming packed FP32 instructions
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", CSRC, "-I", os.path.join(ROOT, "include"),
    "-Wno-unused-result",
]


_PART_IF = re.compile(rb"#(el)?if\s+(MTP_PART\s*==\s*\d+(\s*\|\|\s*MTP_PART\s*==\s*\d+)*)\s*$")


def _part_text(text, part):
    """The lines of a generated kernel file that part `part` compiles: the
    sections under `#if MTP_PART == a || ...` / `#elif` / `#else` are kept
    only where they select `part`; every other line (other conditionals
    included) is kept."""
    out, stack = [], []   # stack entries: [is_part_if, active, taken]
    for line in text.split(b"\n"):
        t = line.strip()
        m = _PART_IF.match(t)
        if m and not m.group(1):
            hit = part in [int(v) for v in re.findall(rb"\d+", m.group(2))]
            stack.append([True, hit, hit])
            continue
        if stack and stack[-1][0]:
            if m and m.group(1):
                hit = part in [int(v) for v in re.findall(rb"\d+", m.group(2))]
                stack[-1][1] = hit and not stack[-1][2]
                stack[-1][2] |= hit
                continue
            if t.startswith(b"#else"):
                stack[-1][1] = not stack[-1][2]
                stack[-1][2] = True
                continue
        if t.startswith((b"#if", b"#ifdef", b"#ifndef")):
            stack.append([False, True, True])
        elif t.startswith(b"#endif"):
            top = stack.pop()
            if top[0]:
                continue
        if all(e[1] for e in stack):
            out.append(line)
    return b"\n".join(out)


def _hash(path, extra):
    h = hashlib.sha256()
    with open(path, "rb") as fh:
        text = fh.read()
    h.update(text)
    # a generated part includes the level's kernel file, of which it compiles
    # only its own sections: a change elsewhere in that file keeps its object
    m = re.search(rb"#define MTP_PART (\d+)", text)
    scanned = text
    for inc in re.findall(rb'#include "(gen_lev\d+\.inc)"', text):
        with open(os.path.join(os.path.dirname(path), inc.decode()), "rb") as fh:
            body = fh.read()
        part = _part_text(body, int(m.group(1))) if m else body
        h.update(part)
        scanned += part
    # the project headers the file includes, directly or through others
    for dep in _includes(scanned):
        with open(dep, "rb") as fh:
            h.update(fh.read())
    h.update(" ".join(extra).encode())
    return h.hexdigest()[:16]


def _includes(text):
    """Paths of the project headers reachable from `text` by #include "..."
    (the generated kernel files themselves excluded), in a fixed order."""
    found, todo = [], [text]
    while todo:
        for name in re.findall(rb'#include "([^"]+)"', todo.pop()):
            name = name.decode()
            if name.startswith("gen_lev"):
                continue
            for d in (CSRC, os.path.join(ROOT, "include")):
                path = os.path.join(d, name)
                if os.path.exists(path) and path not in found:
                    found.append(path)
                    with open(path, "rb") as fh:
                        todo.append(fh.read())
                    break
    return sorted(found)


def _compile(src, force=False):
    base = os.path.splitext(os.path.basename(src))[0]
    tag = _hash(src, FLAGS)
    obj = os.path.join(BUILD, f"{base}.{tag}.o")
    if os.path.exists(obj) and not force:
        return obj, 0.0, "cached"
    t0 = time.time()
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [HIPCC] + FLAGS + lang + ["-c", src, "-o", obj + ".tmp"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{res.stderr[-6000:]}")
    os.replace(obj + ".tmp", obj)
    return obj, time.time() - t0, res.stderr.strip()


def build(levels=None, jobs=None, verbose=True, force=False):
    """Generates, compiles (every source when force, else the changed ones)
    and links the library; returns its path."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(BUILD, exist_ok=True)
    if levels is None:
        # the straight-line bases (levels 2-16) and the table-driven ones
        # (20, 24); MTP_EXTRA_LEVELS (e.g. "18") adds more
        extra = [int(v) for v in os.environ.get("MTP_EXTRA_LEVELS", "").replace(",", " ").split()]
        levels = tuple(sorted(set(codegen.LEVELS) | set(codegen.TABLE_LEVELS) | set(extra)))
    gen_files, _ = codegen.write_all(GEN, levels=levels)
    sources = [os.path.join(CSRC, f) for f in sorted(os.listdir(CSRC)) if f.endswith(".hip")]
    sources += [f for f in gen_files if f.endswith((".hip", ".cpp"))]
    jobs = jobs or min(8, os.cpu_count() or 4)
    objs = []
    # largest generated kernels first so they overlap with the small files
    def cost(p):   # compile the parts of the largest bases first
        size = os.path.getsize(p)
        with open(p, "rb") as fh:
            for inc in re.findall(rb'#include "(gen_lev\d+\.inc)"', fh.read()):
                size += os.path.getsize(os.path.join(os.path.dirname(p), inc.decode()))
        return -size
    sources.sort(key=cost)
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        for obj, dt, msg in ex.map(lambda src: _compile(src, force), sources):
            objs.append(obj)
            if verbose and dt:
                print(f"  compiled {os.path.basename(obj)} in {dt:.1f} s", flush=True)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", "-o", tmp] + objs
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr[-4000:]}")
    os.replace(tmp, LIB)
    # drop stale objects of earlier versions of these sources (objects of
    # sources not in this build, such as levels added by MTP_EXTRA_LEVELS
    # another time, are kept)
    keep = set(os.path.basename(o) for o in objs)
    bases = set(f.split(".")[0] for f in keep)
    for f in os.listdir(BUILD):
        if f.endswith(".o") and f not in keep and f.split(".")[0] in bases:
            os.remove(os.path.join(BUILD, f))
    if verbose:
        print(f"built {LIB}", flush=True)
    return LIB


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=None)
    ap.add_argument("--levels", type=str, default=None)
    ap.add_argument("--force", action="store_true", help="compile every source, ignoring cached objects")
    a = ap.parse_args()
    levels = tuple(int(x) for x in a.levels.split(",")) if a.levels else None
    build(levels=levels, jobs=a.jobs, force=a.force)


if __name__ == "__main__":
    main()
