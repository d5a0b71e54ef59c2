"""MI355X-native DVS event generation (Neurosim's event-simulation hot path).

The compute path is the HIP library ``libnsim_ev.so`` behind the C ABI in
``include/nsim_ev.h``; ``paper_2602_15018_amd.ev`` is its thin Python
binding.  Importing this package loads nothing: the library is opened the
first time an ``EventSim`` is created, and creation fails loudly when it is
missing.
"""

__all__ = ["EventSim", "NsimError"]


def __getattr__(name):
    if name in ("EventSim", "NsimError"):
        from . import ev
        return getattr(ev, name)
    raise AttributeError(name)
