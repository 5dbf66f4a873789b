"""The memory hints reach the machine code (CPU only: hipcc cross-compiles).

A run-time choice between a non-temporal and a plain access of one address is
merged by the optimiser into a plain access, silently; the kernels therefore
take their hints as template parameters.  This test compiles the kernel
sources to gfx950 assembly with the library's own flags and counts the `nt`
cache-policy bits of every stream-collide and adjoint instantiation:
  streaming forward (NT = 1): the 9 loads with c_x = 0 (all loads in the AA
      local step, which reads its own slots) and every store (the periodic
      AA neighbour step of the 4-byte formats has two store sites for each
      direction with c_x != 0: the aligned store of a value parked in LDS
      and the direct store of one whose target lies outside the block);
  cached forward (NT = 0): none;
  streaming adjoint: every PDF and lambda load and every lambda store;
  cached adjoint: none.
It also checks that no packed FP32 arithmetic (v_pk_add_f32, v_pk_mul_f32,
v_pk_fma_f32) appears in any kernel: the build disables the feature.
"""
import os
import re
import subprocess

import pytest

from paper_1803_04937_amd import build as B

KERNEL = re.compile(r'^(_ZN3lbm\d+(k_step_tg|k_step_aa_nb|k_step_aa_loc|k_adjoint_planar|'
                    r'k_adjoint)I\S*?)EEEvNS\S*:\s', re.M)


@pytest.fixture(scope="module")
def assembly(tmp_path_factory):
    """gfx950 assembly of every kernel file, compiled concurrently."""
    d = tmp_path_factory.mktemp("asm")
    procs = {}
    for src in B.SOURCES:
        cmd = [B.HIPCC, *B.FLAGS, "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o",
               str(d / (src + ".s"))]
        procs[src] = subprocess.Popen(cmd, stdout=subprocess.DEVNULL, stderr=subprocess.PIPE)
    out = {}
    for src, p in procs.items():
        _, err = p.communicate(timeout=900)
        assert p.returncode == 0, err.decode()[-2000:]
        out[src] = (d / (src + ".s")).read_text()
    return out


def _counts(asm):
    for m in KERNEL.finditer(asm):
        body = asm[m.end():asm.index(".Lfunc_end", m.end())]
        loads = re.findall(r"global_load\S*[^\n]*", body)
        stores = re.findall(r"global_store\S*[^\n]*", body)
        yield (m.group(1), m.group(2), sum(bool(re.search(r"\bnt\b", x)) for x in loads),
               sum(bool(re.search(r"\bnt\b", x)) for x in stores), len(loads), len(stores))


def test_forward_hints(assembly):
    asm = assembly["step_tg.hip"] + assembly["step_aa.hip"]
    seen = 0
    for name, kind, nl, ns, _, _ in _counts(asm):
        qn, nt = re.search(r"ILi(\d+)E.*ELb([01])$", name).groups()
        qn = int(qn)
        want_l = 0 if nt == "0" else (qn if kind == "k_step_aa_loc" else 9)
        want_s = 0 if nt == "0" else qn
        if kind == "k_step_aa_nb" and nt == "1":
            dt, gen = re.search(r"ILi\d+ELi(\d)ELi\dELb([01])", name).groups()
            if gen == "0" and dt in ("1", "2"):     # FP32, shifted FP32: parked
                want_s += 10 if qn == 19 else 18
        assert (nl, ns) == (want_l, want_s), (name, nl, ns)
        seen += 1
    assert seen > 500, seen


def test_adjoint_hints(assembly):
    asm = assembly["adjoint.hip"]
    seen = 0
    kinds = set()
    for name, kind, nl, ns, n_loads, _ in _counts(asm):
        kinds.add(kind)
        qn = int(re.search(r"ILi(\d+)E", name).group(1))
        gen = re.search(r"ILi\d+ELi\dELi\dELi\dELb([01])", name).group(1) == "1"
        if name.endswith("Lb0"):          # cached policy: no hint at all
            assert nl == 0 and ns == 0, (name, nl, ns)
            seen += 1
            continue
        # every PDF load and every lambda load / store is hinted (without
        # gradients the rest population's PDF is dead: 2 Q - 1 loads); kernels
        # with walls or masks also read the mask and copy lambda through
        # solid cells.  Each direction with c_x != 0 (10 of D3Q19, 18 of
        # D3Q27) has two store sites: the aligned store of a parked push and
        # the direct store of one that could not be parked.
        nxs = 10 if qn == 19 else 18
        assert nl >= 2 * qn - 1 and ns >= qn + nxs, (name, nl, ns)
        if not gen:
            assert nl == n_loads and ns == qn + nxs, (name, nl, n_loads, ns)
        seen += 1
    assert seen > 100, seen
    assert kinds == {"k_adjoint", "k_adjoint_planar"}, kinds


def test_no_packed_fp32(assembly):
    for src, asm in assembly.items():
        hits = re.findall(r"v_pk_(?:add|mul|fma)_f32", asm)
        assert not hits, (src, len(hits))
