"""Seeded synthetic inputs (points, weights, fields) shared by the tests, the
benchmark and the oracle's pins. No convolution arithmetic lives here."""
