"""MI355X-native direct geolocation: the position-domain correlation map and its peak.

Modules
  geoloc   ctypes binding of libgeoloc.so (the gfx950 C-ABI library) and ``Plan``
  sim      seeded scenario simulator (input generator only)
  configs  workload descriptions
  build    hipcc build step of libgeoloc.so

The binding is imported lazily so that the simulator and configs can be used
without a built library; ``geoloc`` itself raises if the library is missing.
"""

__all__ = ["configs", "sim", "geoloc", "build"]
