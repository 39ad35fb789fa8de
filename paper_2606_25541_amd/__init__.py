"""MI355X-native background-field PSFD / Lippmann-Schwinger solver for EUV masks.

``clips``: seeded synthetic inputs. ``api``: torch front end over the HIP
library ``libpsfd.so`` (C ABI in ``include/psfd.h``); the library is loaded
on first use and its absence raises.
"""
from . import clips  # noqa: F401
from . import api  # noqa: F401

__all__ = ["clips", "api"]
