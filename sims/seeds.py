"""Seed discipline: one numpy Generator per (config, stream)."""

import numpy as np

SEED_BASE = 2310_09200

# stream ids: independent draws for each ingredient of an instance
STREAM_LAYOUT = 0
STREAM_SKY = 1
STREAM_NOISE = 2
STREAM_FLAG = 3
STREAM_WEIGHTS = 4
STREAM_EIG = 5


def rng(config_id, stream_id, *extra):
    """Generator seeded by ``SeedSequence([SEED_BASE, config_id, stream_id, *extra])``."""
    ent = [SEED_BASE, int(config_id), int(stream_id)] + [int(e) for e in extra]
    return np.random.default_rng(np.random.SeedSequence(ent))
