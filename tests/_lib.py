"""Test helpers: load the built libspx (building it once if nothing is built yet)."""
import os

import paper_2502_19284_amd as spx
from paper_2502_19284_amd import build as spx_build


def ensure_built():
    if not os.path.exists(spx.LIB_PATH):
        spx_build.build()
    return spx.load()
