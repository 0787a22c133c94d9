"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

Holds no solver arithmetic: it only builds the block-sparse systems the
solver consumes (see ``generator``)."""
from .generator import (BSRSystem, P_INDEX, T_INDEX, assemble, tiny, config1, config2,
                        config3, config4_train, config5, config5_field, named,
                        CONFIG2_PECLET, CONFIG3_PECLET)
from .mlp_init import mlp_init
from .full_system import FullSystem, Wells, full_system, wells
