"""Machine descriptors for the case-table tests (no GPU needed).

* gfx950: the hipDeviceProp_t fields recorded on an MI355X
  (tests/golden/gfx950_props.json);
* mi300x_like: 64 KiB LDS per workgroup (CDNA3), otherwise as gfx950;
* fermi_like: 48 KiB shared memory, 32768 registers per block, 1024 threads;
* the enumerator's grid of LDS / register / thread limits.
"""
import json
import os

from paper_1801_04348_amd import pk

_GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "gfx950_props.json")


def gfx950():
    with open(_GOLDEN) as f:
        p = json.load(f)["props"]
    return pk.machine(wave=p["warpSize"], lds_block=p["sharedMemPerBlock"],
                      lds_cu=p["maxSharedMemoryPerMultiProcessor"], regs_block=p["regsPerBlock"],
                      regs_cu=p["regsPerMultiprocessor"], max_threads_block=p["maxThreadsPerBlock"],
                      max_threads_cu=p["maxThreadsPerMultiProcessor"],
                      max_blocks_cu=p["maxBlocksPerMultiProcessor"], cu_count=p["multiProcessorCount"],
                      clock_khz=p["clockRate"], arch=p["gcnArchName"])


def variant(base=None, **kw):
    m = base or gfx950()
    d = m.as_dict()
    d.update(kw)
    return pk.machine(**d)


def mi300x_like():
    return variant(lds_block=65536, lds_cu=65536, cu_count=304, clock_khz=2100000, arch="gfx942-like")


def fermi_like():
    return variant(wave=32, lds_block=49152, lds_cu=49152, regs_block=32768, regs_cu=32768,
                   max_threads_block=1024, max_threads_cu=1536, max_blocks_cu=8, cu_count=14,
                   clock_khz=1150000, arch="fermi-like")


def grid_machine(Z, V, T):
    return variant(lds_block=Z, lds_cu=max(Z, 65536), regs_block=V, regs_cu=max(V, 65536), max_threads_block=T)
