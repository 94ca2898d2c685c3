"""MI355X (gfx950) X-engine correlator: 4+4-bit complex samples in, exact
int32 upper-triangle visibilities out (the correlation task of the CHIME GPU
X-engine, Sec. 2.2 and Sec. 3.1 of the paper)."""
from .xeng import (  # noqa: F401
    Batch, Correlator, Server, Tuning, XengError, autotune, clock_probe, correlate_batch, dump_batch,
    correlate_reference, max_integration, plan_inspect, sclk_ghz, set_tuning, slot_bytes, tri,
)
