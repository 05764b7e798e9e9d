"""Compile the library's kernel source for the CPU (tests only).

The HIP kernel file is rewritten mechanically -- the dynamic LDS array becomes
the emulated workgroup's buffer, inline assembly (waits and compiler fences)
becomes a wave reconvergence barrier, the HIP launch wrappers are dropped --
and compiled with g++ against hip/hip_runtime.h from this directory.
"""
import os
import re
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
CSRC = os.path.join(ROOT, "paper_2602_10080_amd", "csrc")
KERNEL = os.path.join(CSRC, "mlmq_kernels.hip")


def transformed_source(checked: bool = False) -> str:
    src = open(KERNEL).read()
    if checked:
        # bounds-check every edge and vertex index the kernel dereferences
        src = src.replace("c.q.adj[eidx]", "c.q.adj[simt_chk(eidx, (uint64_t)c.q.off[c.q.n], \"adj\", __LINE__)]")
        src = src.replace("c.q.off[lv]", "c.q.off[simt_chk(lv, c.q.n, \"off\", __LINE__)]")
        src = src.replace("c.q.dist + lv", "c.q.dist + simt_chk(lv, c.q.n, \"dist\", __LINE__)")
        src = src.replace("c.q.dist + v[u]", "c.q.dist + simt_chk(v[u], c.q.n, \"dist\", __LINE__)")
        src = src.replace("c.q.dist + hv", "c.q.dist + simt_chk(hv, c.q.n, \"dist\", __LINE__)")
        src = src.replace("ld_label(c.q.dist + v)", "ld_label(c.q.dist + simt_chk(v, c.q.n, \"dist\", __LINE__))")
        # optimality check kernels
        chk = [("(uint32_t)off[p]", "(uint32_t)off[simt_chk(p, n + 1u, \"off\", __LINE__)]"),
               ("off[min(r + lane() + 1u, n)]", "off[simt_chk(min(r + lane() + 1u, n), n + 1u, \"off\", __LINE__)]"),
               ("dist[r + j]", "dist[simt_chk(r + j, n, \"dist\", __LINE__)]"),
               ("const uint64_t a = adj[e];", "const uint64_t a = adj[simt_chk(e, m, \"adj\", __LINE__)];"),
               ("dist[(uint32_t)a]", "dist[simt_chk((uint32_t)a, n, \"dist\", __LINE__)]"),
               ("tight[(uint32_t)a]", "tight[simt_chk((uint32_t)a, n, \"tight\", __LINE__)]"),
               ("const uint32_t d = dist[v];", "const uint32_t d = dist[simt_chk(v, n, \"dist\", __LINE__)];"),
               ("tight[v] == 0", "tight[simt_chk(v, n, \"tight\", __LINE__)] == 0")]
        for a, b in chk:
            src = src.replace(a, b)
        for pat in ("c.q.adj[eidx]", "c.q.off[lv]", "c.q.dist + lv", "c.q.dist + v[u]", "c.q.dist + hv",
                    "ld_label(c.q.dist + v)", *[a for a, _ in chk]):
            assert pat in open(KERNEL).read(), pat
    src = src.replace("extern __shared__ uint64_t smem[];",
                      "uint64_t* smem = reinterpret_cast<uint64_t*>(simt::group->lds);")
    src = re.sub(r'asm volatile\("([^"]*)"\s*:::\s*"memory"\);', lambda mo: 'simt::wave_sync_at("asm ' + mo.group(1) + '");', src)
    cut = src.index("hipError_t launch_init(")
    return src[:cut] + "\n}  // namespace mlmq\n"


def build(out_dir: str, sanitize: bool = False, checked: bool = True) -> str:
    """Builds into a directory of this process's own, then moves the library
    into place (parallel test workers may build at the same time)."""
    work = os.path.join(out_dir, "tmp%d" % os.getpid())
    os.makedirs(work, exist_ok=True)
    with open(os.path.join(work, "sim_kernels.inc"), "w") as f:
        f.write(transformed_source(checked))
    lib = os.path.join(out_dir, "libsim%s.so" % ("_asan" if sanitize else ""))
    tmp = os.path.join(work, os.path.basename(lib))
    cmd = ["g++", "-std=c++20", "-O1", "-g", "-fPIC", "-shared", "-pthread", "-w",
           "-I", HERE, "-iquote", CSRC, "-iquote", work,
           os.path.join(HERE, "harness.cpp"), "-o", tmp]
    if sanitize:
        cmd[1:1] = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer"]
    subprocess.check_call(cmd)
    os.replace(tmp, lib)
    os.remove(os.path.join(work, "sim_kernels.inc"))
    os.rmdir(work)
    return lib


if __name__ == "__main__":
    print(build(os.path.join(ROOT, "_build", "simt")))
