"""Plants one plausible mistake at a time in a private build of the oracle
and checks that the pins catch each one.  This shows the pins are sharp
enough that a wrong oracle cannot pass them.  Everything here runs on the
CPU, on copies of the oracle built into a temporary directory.
"""
import os

import pytest

from oracle import build, ref
from tests import pins

PLANTS = {
    "REF_PLANT_XTIME": "xtime without reduction",
    "REF_PLANT_AFFINE": "S-box affine constant wrong",
    "REF_PLANT_SHIFTROWS": "ShiftRows rotates the wrong way",
    "REF_PLANT_MIXCOL": "MixColumns coefficient {03} read as {01}",
    "REF_PLANT_RCON": "Rcon dropped from KeyExpansion",
    "REF_PLANT_LASTKEY": "final AddRoundKey dropped",
    "REF_PLANT_CTR_LE": "CTR counter stored little-endian",
    "REF_PLANT_CBC_PLAIN": "CBC chains the previous plaintext instead of the ciphertext",
    "REF_PLANT_XTS_NOREDUCE": "XTS tweak doubling without the reduction",
    "REF_PLANT_XTS_BE": "XTS tweak value written as a big-endian number",
    "REF_PLANT_GCM_R": "GHASH reduction constant at the wrong end of the block",
    "REF_PLANT_GCM_LEN": "GCM length block counts bytes instead of bits",
}


@pytest.mark.parametrize("macro", sorted(PLANTS))
def test_pins_catch_planted_mistake(tmp_path, macro):
    lib = build.build(os.path.join(str(tmp_path), "liboracle_%s.so" % macro), defines=[macro])
    mutant = ref.Oracle(lib)
    results = pins.run_all(mutant)
    failed = [name for name, f in results.items() if f]
    assert failed, "no pin caught: " + PLANTS[macro]


def test_clean_build_passes_all_pins(tmp_path):
    lib = build.build(os.path.join(str(tmp_path), "liboracle_clean.so"))
    results = pins.run_all(ref.Oracle(lib))
    assert all(not f for f in results.values()), results
