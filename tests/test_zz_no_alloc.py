"""The entry point that allocates nothing (nqs_local_energy_noalloc, for callers
that cannot allocate device memory) against nqs_local_energy: bit for bit on two
calls in a row, the second with a smaller batch, for each precision and both
Hamiltonian kinds; batches beyond the static scratch are rejected."""
import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a visible HIP device")
    return torch


CASES = [
    ("tfim2d_l10", "fp64", 16384, 3001),   # full batch of the 10x10 workload, then a ragged one
    ("tfim2d_l10", "bf16", 5000, 333),
    ("heis1d_n64", "fp32", 4099, 1000),
    ("heis2d_l16", "bf16", 2048, 65),
]


@pytest.mark.parametrize("name,precision,n1,n2", CASES)
def test_noalloc_matches_local_energy(name, precision, n1, n2):
    torch = _torch()
    from paper_2112_10526_amd.nqs import VMCState
    print(f"[case] {name} {precision} n={n1},{n2}", flush=True)
    w = synth.WORKLOADS[name].replace(sigma=0.05, n_chains=min(synth.WORKLOADS[name].n_chains, 2048))
    st = VMCState.from_workload(w, precision=precision)
    gen = synth.sz0_configs if w.total_sz_zero else synth.random_configs
    for n, seed in ((n1, 21), (n2, 22)):
        s = torch.from_numpy(gen(n, w.n_sites, seed)).to("cuda")
        ref = st.local_energy(s)
        out = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        st.local_energy_noalloc(s, out)
        torch.cuda.synchronize()
        a, b = ref.cpu().numpy(), out.cpu().numpy()
        assert np.isfinite(a).all()
        np.testing.assert_array_equal(b, a)
    st.close()


def test_noalloc_rejects_batches_beyond_scratch():
    torch = _torch()
    from paper_2112_10526_amd._lib import NQS_EINVAL, NqsError
    from paper_2112_10526_amd.nqs import VMCState
    w = synth.WORKLOADS["tfim2d_l10"].replace(n_chains=64, samples_per_chain=1)
    st = VMCState.from_workload(w, precision="fp64")
    n = 32769  # 32,769 x 256 activations x 8 B > 64 MiB
    s = torch.ones((n, w.n_sites), dtype=torch.int8, device="cuda")
    out = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(NqsError) as e:
        st.local_energy_noalloc(s, out)
    assert e.value.status == NQS_EINVAL and "static scratch" in str(e.value)
    assert float(out.abs().sum()) == 0.0  # nothing was written
    st.local_energy_noalloc(s[:32768], out)  # the largest batch that fits
    ref = st.local_energy(s[:32768])
    np.testing.assert_array_equal(out[:32768].cpu().numpy(), ref.cpu().numpy())
    st.close()
