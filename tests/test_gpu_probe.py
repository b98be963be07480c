"""GPU: the device-rate probes (pimm_probe) return plausible rates.

They are measurement tools, so the checks are sanity bounds: positive rates below
the published MI355X peaks, and the FP64 modular product (the form the library
uses) faster than the 64-bit integer Barrett form."""
import pytest
import torch

from paper_2305_18396_amd import pimm

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no HIP device", allow_module_level=True)


def test_memory_probes_below_peak():
    for kind in (pimm.PROBE_READ, pimm.PROBE_READ8, pimm.PROBE_COPY):
        rate = pimm.probe(kind, 256 << 20, reps=2)
        assert 1e11 < rate < 8.5e12, (kind, rate)


def test_arithmetic_probes():
    fma = pimm.probe(pimm.PROBE_FMA64, 1024, reps=1)
    assert 1e12 < fma < 80e12
    f64 = pimm.probe(pimm.PROBE_MODMUL_F64, 1024, reps=1)
    barrett = pimm.probe(pimm.PROBE_MODMUL_BARRETT, 1024, reps=1)
    shoup = pimm.probe(pimm.PROBE_MODMUL_SHOUP, 1024, reps=1)
    assert f64 > barrett > 0 and shoup > 0
