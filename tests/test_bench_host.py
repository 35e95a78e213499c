"""Host-side accounting of bench.py (CPU): the algorithmic vector passes behind
`roofline.achieved`, and the lookup of the committed traffic counters."""
import pytest

import bench


@pytest.mark.parametrize("l", range(1, 9))
def test_plcg_vector_passes(l):
    # reads: z_i, z_{i-1}, 2 per basis k < l, max(0, l-3) older z, p_{t-1};
    # writes: z_{i+1}, l basis vectors, p_t -> 3l + 5 + max(0, l-3); x adds 2
    # (read + write every sweep) or 1.5 (x and p_{t-2} read, x written, every
    # second sweep)
    base = 3 * l + 5 + max(0, l - 3)
    assert bench.vector_passes("plcg", l, 1) == base + 2
    assert bench.vector_passes("plcg", l, 2) == base + 1.5
    assert bench.vector_passes("plcg", l) == base + 2     # default: every sweep


def test_cg_vector_passes():
    # sweep A: r, p_{k-1} in, p_k, A p_k out (4); sweep B: x, p, r, A p in,
    # x, r out (6), or alternately 3 (r, A p in, r out) and 7 (+ x, p_k,
    # p_{k-1} in, x out)
    assert bench.vector_passes("cg", 1, 1) == 4 + 6
    assert bench.vector_passes("cg", 1, 2) == 4 + (3 + 7) / 2


def test_headline_bytes_per_iteration():
    # 2048^2 FP64 p(1)-CG with paired x updates: 9.5 vectors of 2^22 doubles
    n = 2048 * 2048
    assert bench.vector_passes("plcg", 1, 2) * 8 * n == 318767104


def test_measured_traffic_lookup():
    got = bench.measured_traffic("poisson2048", "plcg_sweep_kernel<1,false,double>")
    if got is None:
        pytest.skip("counter summary older than the kernel sources")
    name, b = got
    assert name.startswith("plcg_sweep_kernel<1,false,double,")
    # the counters agree with the algorithmic bytes to within 1 %
    assert abs(b / 318767104 - 1) < 0.01
    assert bench.measured_traffic("poisson2048", "no_such_kernel<1>") is None


def test_working_set_and_cache_residency():
    """The 2048^2 p(1)-CG sweep (paired x updates) touches 7 vectors of 32 MiB:
    2 of basis 0, 2 ring slots, 2 p buffers and x = 224 MiB, inside the 256 MiB
    memory-side cache; 256^3 p(3)-CG touches 11 vectors of 128 MiB."""
    n2 = 2048 * 2048
    assert bench.working_set("plcg", 1, 2, n2, 8, 0) == 7 * 8 * n2 <= bench.CACHE_BYTES
    assert bench.working_set("plcg", 1, 1, n2, 8, 0) == 6 * 8 * n2
    assert bench.working_set("cg", 0, 2, n2, 8, 0) == 5 * 8 * n2
    n3 = 256 ** 3
    assert bench.working_set("plcg", 3, 2, n3, 8, 0) == 11 * 8 * n3 > bench.CACHE_BYTES
    assert bench.working_set("plcg", 5, 1, n3, 4, 0) == (10 + 4 + 1 + 1) * 4 * n3


def test_kernel_source_hash_ignores_comments_and_layout():
    """The hash that ties the committed traffic counters to the kernels it was
    taken with covers the code only: comments and layout may change, code not."""
    import bench
    src = ('int a = 1; // one\n/* two\n lines */ double b = "x//y /* z */";\n'
           "char q = '/';   // end\n  int   c = a*2;")
    assert bench.code_only(src) == 'int a = 1; double b = "x//y /* z */"; char q = \'/\'; int c = a*2;'
    commented = "// header\nint f(int x) {  /* doubled */\n  return 2 * x;   // here\n}\n"
    plain = "int f(int x) { return 2 * x; }"
    assert bench.code_only(commented) == bench.code_only(plain)
    assert bench.code_only(plain) != bench.code_only(plain.replace("2", "3"))
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()
