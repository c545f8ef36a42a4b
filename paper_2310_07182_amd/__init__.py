"""MI355X-native secondary-ray path tracer with coherent direction reuse
("Generate Coherent Rays Directly", Liu et al., EG 2024)."""
