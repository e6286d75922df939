"""Observation digests for parity tests that compare every game's
observations every ply without copying them to the host: the digest of a
block of bytes is the sum of byte i times w(i) modulo 2^64, w(i) the
SplitMix64 output for the counter value i + 1.  The oracle library forms it
in C (oracle.digest_blocks); this module forms the same sum in numpy (to pin
the C one) and on the device with torch."""
import numpy as np


def weights(block):
    i = np.arange(1, block + 1, dtype=np.uint64)
    z = i * np.uint64(0x9E3779B97F4A7C15)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def digest_numpy(blocks):
    """blocks: uint8 [m, block] -> uint64 [m]."""
    b = np.asarray(blocks, dtype=np.uint8)
    w = weights(b.shape[1])
    return (b.astype(np.uint64) * w).sum(axis=1, dtype=np.uint64)


class DeviceDigest:
    """The same digest of uint8 [m, block] GPU tensors, with int64 arithmetic
    (wrapping modulo 2^64 like the unsigned sums), in row chunks."""

    def __init__(self, torch, block, device="cuda", rows_per_chunk=1024):
        self.torch = torch
        self.block = block
        self.w = torch.from_numpy(weights(block).view(np.int64)).to(device)
        self.rows = rows_per_chunk

    def __call__(self, blocks):
        torch = self.torch
        b = blocks.reshape(-1, self.block)
        out = torch.empty(b.shape[0], dtype=torch.int64, device=b.device)
        for s in range(0, b.shape[0], self.rows):
            out[s:s + self.rows] = (b[s:s + self.rows].to(torch.int64) * self.w).sum(dim=1)
        return out.cpu().numpy().view(np.uint64)
