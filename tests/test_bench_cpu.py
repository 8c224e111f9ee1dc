"""CPU checks of the benchmark's own arithmetic and bookkeeping: the algorithmic
work it divides by for the roofline, the lookup of committed counter summaries,
and the single-GPU contract.  No GPU needed."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def ntt(n):
    # butterflies of one transform of n residues, one modular product each
    return (n // 2) * (n.bit_length() - 1)


def test_modmul_counts_closed_forms():
    """Per pair at n = 16384, L = 7: the plain inner-product launch counts the
    L (L - 1) digit transforms, the special prime's L transforms, 2 L n products
    per target modulus and two inverse transforms with their n^-1 scaling; the
    split variant's data-modulus launch counts, per data modulus, L - 1 digit
    transforms, 2 L n products, rho's two transforms and 2 n products by P^-1."""
    n, L = 16384, 7
    assert ntt(n) == 114688
    plain = L * ((L - 1) * ntt(n) + 2 * L * n) + (L * ntt(n) + 2 * L * n + 2 * (ntt(n) + n))
    assert plain == 7716864 == bench.ks_mac_modmuls(n, L, 1)
    md = L * ((L - 1) * ntt(n) + 2 * L * n + 2 * ntt(n) + 2 * n)
    assert md == 8257536 == bench.ks_mac_md_modmuls(n, L, 1)
    for pairs in (1, 16, 4096):
        assert bench.ks_mac_modmuls(n, L, pairs) == pairs * plain
        assert bench.ks_mac_md_modmuls(n, L, pairs) == pairs * md
    # the paper's ring at its L = 6: the same forms
    assert bench.ks_mac_md_modmuls(8192, 6, 1) == 6 * (5 * ntt(8192) + 2 * 6 * 8192 + 2 * ntt(8192) + 2 * 8192)


def test_counted_traffic_needs_matching_sources_and_variant(tmp_path, monkeypatch):
    """A committed counter summary is used only for its own launch variant and
    only while the kernel sources hash to the digest it records."""
    digest = bench.kernel_source_digest()
    assert len(digest) == 64 and int(digest, 16) >= 0
    path = tmp_path / "k_ks_mac_traffic_batch_512x40000x16_le{le}_mode{mode}.txt"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))
    body = "kernel_source_sha256: {d}\nle_mac: 6\nmac_mode: 6\ntraffic_bytes_per_launch: 123456789\n"
    (tmp_path / "k_ks_mac_traffic_batch_512x40000x16_le6_mode6.txt").write_text(body.format(d=digest))
    assert bench.counted_traffic(6, 6) == 123456789
    assert bench.counted_traffic(5, 6) is None          # no summary for that variant
    (tmp_path / "k_ks_mac_traffic_batch_512x40000x16_le6_mode6.txt").write_text(body.format(d="0" * 64))
    assert bench.counted_traffic(6, 6) is None          # sources changed since the counters were taken


@pytest.mark.parametrize("le_mac,mac_mode", [(6, 6), (5, 6), (4, 7)])
def test_committed_traffic_summaries_are_current(le_mac, mac_mode):
    """The summaries for the large-tile choices the autotuner has picked match the
    committed kernel sources (the benchmark's roofline traffic field reads them)."""
    assert bench.counted_traffic(le_mac, mac_mode) is not None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
