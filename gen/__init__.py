"""Seeded synthetic inputs shared by the oracle tests and the HIP path.

Holds geometry and random numbers only, none of the contact method's
arithmetic."""
