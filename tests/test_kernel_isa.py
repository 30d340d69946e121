"""Static checks of the gfx950 code the compiler emits for the persistent
kernels of the co-execution, batched and serving forms (CPU only: hipcc
cross-compiles).

A workgroup barrier inside a loop whose exit is decided per lane (an exec-mask
update followed by a branch on an empty mask) lets some lanes leave the loop
while the rest of the wave keeps executing the barrier; the workgroup then
never makes progress. The persistent loops are written so that every branch
around a barrier is uniform; this test keeps it that way."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1805_02755_amd", "csrc")
HIPCC = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
# source file -> (kernel name fragment, number of instantiations) for each
# kernel with a tile loop: the persistent kernels and the direct kernels of
# the co-execution, the batched and the serving forms
SOURCES = {"kernels.hip": (("k_persistent", 7), ("k_direct", 7)), "batch_kernels.hip": (("k_batch_escape", 5),),
           "serve_kernels.hip": (("k_serve", 1),)}


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    d = tmp_path_factory.mktemp("isa")
    texts = {}
    for src in SOURCES:
        out = d / (src + ".s")
        cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-ffp-contract=off", "-Xclang",
               "-target-feature", "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-S", "-o", str(out),
               os.path.join(CSRC, src)]
        subprocess.run(cmd, check=True, capture_output=True)
        texts[src] = out.read_text()
    return texts


def _functions(text):
    funcs = {}
    for m in re.finditer(r"^(_Z\w+):.*?$(.*?)^\s*s_endpgm", text, flags=re.S | re.M):
        funcs[m.group(1)] = m.group(2)
    return funcs


def _blocks(body):
    """(label, loop header or None, lines) per basic block."""
    blocks = []
    cur = None
    for ln in body.splitlines():
        m = re.match(r"^(\.LBB\w+|; %bb\.\d+):(.*)$", ln)
        if m:
            hdr = re.search(r"Header=(BB\w+)", m.group(2))
            own = re.search(r"This (?:Inner )?Loop Header", m.group(2))
            label = m.group(1).lstrip(".").removeprefix("L")
            cur = [label, hdr.group(1) if hdr else (label if own else None), []]
            blocks.append(cur)
            continue
        if "This Loop Header" in ln or "This Inner Loop Header" in ln:
            if cur is not None and cur[1] is None:
                cur[1] = cur[0]
        if cur is not None:
            cur[2].append(ln.strip())
    return blocks


@pytest.mark.parametrize("src", sorted(SOURCES))
def test_persistent_loops_have_uniform_exits_around_barriers(asm, src):
    funcs = {}
    for frag, count in SOURCES[src]:
        these = {k: v for k, v in _functions(asm[src]).items() if frag in k}
        assert len(these) == count, (frag, sorted(these))
        funcs.update(these)
    for name, body in funcs.items():
        blocks = _blocks(body)
        barrier_loops = {hdr for _, hdr, lines in blocks if hdr and any(l.startswith("s_barrier") for l in lines)}
        for label, hdr, lines in blocks:
            if hdr not in barrier_loops:
                continue
            txt = "\n".join(lines)
            bad = re.search(r"s_andn2_b64 exec, exec, s\[\d+:\d+\]\s*\n\s*s_cbranch_execz", txt)
            assert not bad, f"{name}: loop {hdr} holds a barrier and a per-lane exit in {label}"


@pytest.mark.parametrize("src", sorted(SOURCES))
def test_no_packed_fp32_and_no_spills(asm, src):
    for name, body in _functions(asm[src]).items():
        for op in ("v_pk_fma_f32", "v_pk_mul_f32", "v_pk_add_f32"):
            assert op not in body, (name, op)
    assert "scratch_store" not in asm[src]


def test_serving_kernel_drops_stale_lines_at_job_switch(asm):
    """Inputs copied in during a session are read after a system-scope
    invalidate (the job-switch acquire)."""
    body = next(v for k, v in _functions(asm["serve_kernels.hip"]).items() if "k_serve" in k)
    assert "buffer_inv sc0 sc1" in body


def _kernel_meta(text):
    """name -> (argument (offset, size) list, private segment bytes) from the
    code object's kernel metadata."""
    meta = {}
    for m in re.finditer(r"\.args:\s*\n(.*?)\n    \.group_segment_fixed_size.*?\.name:\s+(\S+)\n(.*?)(?=\n  - \.|\n\.end_amdgpu_metadata)",
                         text, flags=re.S):
        args = [(int(o), int(s)) for o, s in re.findall(r"\.offset:\s+(\d+)\s*\n\s*\.size:\s+(\d+)", m.group(1))]
        priv = re.search(r"\.private_segment_fixed_size:\s+(\d+)", m.group(3))
        meta[m.group(2)] = (args, int(priv.group(1)) if priv else None)
    return meta


def test_persistent_kernel_reads_its_arguments_where_the_abi_puts_them(asm):
    """The persistent kernel copies its scheduler arguments into LDS from the
    kernel-argument segment at the offset the payload's size and the block's
    alignment give; the metadata must place the block there, for every
    payload. No tile kernel uses scratch memory."""
    meta = _kernel_meta(asm["kernels.hip"])
    seen = 0
    for name, (args, priv) in meta.items():
        if "k_persistent" not in name and "k_direct" not in name:
            continue
        assert priv == 0, (name, priv)
        if "k_persistent" in name:
            (o0, s0), (o1, s1) = args[0], args[1]
            assert o0 == 0 and o1 == (s0 + 7) // 8 * 8, (name, args[:2])
            seen += 1
    assert seen == 7


def test_persistent_kernel_starts_without_waiting_on_its_arguments(asm):
    """Only the few arguments of the direct phase are loaded before the first
    branch: at most two waits on scalar loads, where loading the whole block
    at the entry took four and spilled registers."""
    for name, body in _functions(asm["kernels.hip"]).items():
        if "k_persistent" not in name:
            continue
        lines = [l.strip() for l in body.splitlines()]
        entry = []
        for l in lines:
            if l.startswith("s_cbranch"):
                break
            entry.append(l)
        assert sum(l.startswith("s_waitcnt lgkmcnt(0)") for l in entry) <= 2, name


def test_nbody_loop_reads_each_batch_a_phase_ahead(asm):
    """The n-body inner loop keeps two batches of eight bodies: after issuing
    a batch's eight LDS reads, it computes the batch read before, so until
    the next reads no wait may reach into the batch just issued (lgkmcnt
    stays at 8 or more). Otherwise the reads' latency would wait on the
    arithmetic, with one wave per SIMD to hide it."""
    seen = 0
    for src in ("kernels.hip",):
        for name, body in _functions(asm[src]).items():
            if "Nbody" not in name:
                continue
            for block in re.split(r"\n(?=\.LBB\d+_\d+:)", body):
                lines = [l.strip() for l in block.splitlines()]
                if sum(l.startswith("ds_read_b128") for l in lines) != 16:
                    continue
                after_batch = False
                for l in lines:
                    if l.startswith("ds_read_b128"):
                        after_batch = True
                        continue
                    m = re.match(r"s_waitcnt lgkmcnt\((\d+)\)", l)
                    if m and after_batch:
                        assert int(m.group(1)) >= 8, (name, l)
                seen += 1
    assert seen >= 16
