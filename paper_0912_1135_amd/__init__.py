"""MI355X-native randomized orthogonal projection (Rokhlin & Tygert)."""
