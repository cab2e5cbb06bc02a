"""FP64 CPU oracle of FPS-SFT. Test infrastructure: imported only by tests,
the smoke check and the benchmark's CPU-baseline leg."""
from .fpssft_oracle import *  # noqa: F401,F403
from .fpssft_oracle import (Params, Result, run, schedule, replay_amplitudes,  # noqa: F401
                            STATUS_OK, STATUS_INCOMPLETE, STATUS_CAPACITY)
