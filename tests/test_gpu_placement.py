"""GPU: where the reaction parameters live (registers, LDS, global memory) never
changes a result: the kernels run the same arithmetic in the same order, so
the placements agree bit for bit; the global-memory variant is also checked
against the oracle, and asking for a placement without a compiled variant is
an error."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1309_2710_amd import synth
from tests import parity as PT

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def R():
    from paper_1309_2710_amd import rkc
    rkc.lib()
    return rkc


def _say(*a):
    print("[case]", *a, flush=True)


def _run(R, gm, cfg, st, placement):
    c = synth.CONFIGS[cfg]
    T, Y = st["T"].copy(), st["Y"].copy()
    out = R.integrate(gm, T, st["P"], Y, c["dt"], c["rtol"], c["atol"], counters=True,
                      stats=True, param_placement=placement)
    return T, Y, out


def test_global_tables_equal_lds_and_oracle(R):
    """111 species: the LDS tables limit the workgroup, so the automatic choice
    reads the parameters from global memory; both placements agree bit for
    bit and match the oracle."""
    _say("placement c4")
    m = synth.config_mechanism("c4")
    gm = R.Mechanism(m)
    st = synth.config_states("c4", 24)
    Tl, Yl, ol = _run(R, gm, "c4", st, R.PARAMS_LDS)
    Tg, Yg, og = _run(R, gm, "c4", st, R.PARAMS_GLOBAL)
    Ta, Ya, oa = _run(R, gm, "c4", st, R.PARAMS_AUTO)
    _say("lds", ol["stats"], "global", og["stats"], "auto", oa["stats"])
    for T, Y, o in ((Tg, Yg, og), (Ta, Ya, oa)):
        assert np.array_equal(Tl, T) and np.array_equal(Yl, Y)
        assert np.array_equal(ol["counters"], o["counters"])
    assert og["stats"]["lds_bytes"] < ol["stats"]["lds_bytes"]
    assert oa["stats"]["lds_bytes"] == og["stats"]["lds_bytes"]
    assert og["stats"]["block_threads"] > ol["stats"]["block_threads"]
    c = synth.CONFIGS["c4"]
    To, Yo, co = O.Model(m).integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                                      threads=16)
    PT.check(Tg, Yg, og["counters"], To, Yo, co, c["rtol"], c["atol"], PT.max_flips("c4", 24),
             long_set=True)


def test_global_tables_with_falloff(R):
    """The pressure-dependent kernels of the global-memory placement: the
    111-species set with third-body and falloff pairs, global against LDS bit
    for bit and against the oracle."""
    _say("placement c4p")
    m = synth.config_mechanism("c4p")
    gm = R.Mechanism(m)
    st = synth.config_states("c4p", 12)
    Tl, Yl, ol = _run(R, gm, "c4p", st, R.PARAMS_LDS)
    Tg, Yg, og = _run(R, gm, "c4p", st, R.PARAMS_GLOBAL)
    _say("lds", ol["stats"], "global", og["stats"])
    assert np.array_equal(Tl, Tg) and np.array_equal(Yl, Yg)
    assert np.array_equal(ol["counters"], og["counters"])
    c = synth.CONFIGS["c4p"]
    To, Yo, co = O.Model(m).integrate(st["T"], st["P"], st["Y"], c["dt"], c["rtol"], c["atol"],
                                      threads=16)
    PT.check(Tg, Yg, og["counters"], To, Yo, co, c["rtol"], c["atol"], PT.max_flips("c4p", 12),
             long_set=True)


def test_registers_equal_lds(R):
    _say("placement registers c3")
    m = synth.config_mechanism("c3")
    gm = R.Mechanism(m)
    st = synth.config_states("c3", 40)
    Tl, Yl, ol = _run(R, gm, "c3", st, R.PARAMS_LDS)
    Tr, Yr, orr = _run(R, gm, "c3", st, R.PARAMS_REGISTERS)
    assert np.array_equal(Tl, Tr) and np.array_equal(Yl, Yr)
    assert np.array_equal(ol["counters"], orr["counters"])


def test_global_without_variant_is_an_error(R):
    _say("placement global unsupported c3")
    gm = R.Mechanism(synth.config_mechanism("c3"))
    st = synth.config_states("c3", 8)
    with pytest.raises(R.RkcError):
        _run(R, gm, "c3", st, R.PARAMS_GLOBAL)
