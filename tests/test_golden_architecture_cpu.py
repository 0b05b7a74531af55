"""The paper-scale deblurring network against the architecture the paper
specifies (its appendix table and network subsection, transcribed in
tests/golden/unet_architecture.txt): every block's convolutions, the
transposed convolutions that halve the channels, the skip concatenation
that doubles a decoder block's input, the 1x1 output layer, and the
configuration the FWI driver runs as the paper's network."""
import os

from synth import netparams
from paper_2403_17518_amd import fwi_driver

HERE = os.path.dirname(os.path.abspath(__file__))


def _fixture():
    blocks, scalars = [], {}
    with open(os.path.join(HERE, "golden", "unet_architecture.txt")) as f:
        for line in f:
            line = line.split("#", 1)[0].split()
            if len(line) == 5:
                blocks.append((line[0], line[1], int(line[2]), int(line[3]), int(line[4])))
            elif len(line) == 2:
                scalars[line[0]] = float(line[1])
    return blocks, scalars


def test_fixture_is_the_table():
    blocks, scalars = _fixture()
    assert [b[0] for b in blocks] == ["input", "down1", "down2", "down3", "down4",
                                      "up1", "up2", "up3", "up4", "output"]
    assert scalars == {"leaky_slope": 0.2, "pool_kernel": 3, "pool_stride": 2, "input_channels": 1}


def test_paper_network_matches_the_table():
    blocks, scalars = _fixture()
    depth = sum(1 for b in blocks if b[1] == "avgpool")
    base = blocks[0][4]
    assert fwi_driver.NETWORKS["paper"] == (depth, base, scalars["leaky_slope"])
    shapes = dict(netparams.param_shapes(depth, base))
    prev = int(scalars["input_channels"])
    n_up = 0
    for name, opens, nconv, k, ch in blocks:
        if name == "input":
            key = "inc"
        elif opens == "avgpool":
            key = "down" + name[4:]
        elif opens == "convtranspose":
            # the decoder's blocks are numbered from the bottom in the library
            key = f"up{depth - 1 - n_up}"
            n_up += 1
            # a 2x2 stride-2 transposed convolution halving the channels
            assert shapes[key + ".wt"] == (prev, prev // 2, 2, 2) and prev // 2 == ch, name
            assert shapes[key + ".bt"] == (ch,)
        else:
            assert nconv == 1 and k == 1
            assert shapes["outc.w"] == (ch, prev, 1, 1) and shapes["outc.b"] == (ch,)
            prev = ch
            continue
        assert nconv == 2
        # first convolution: the previous block's channels (a decoder block
        # also takes the encoder's skip connection: twice its own width)
        cin = 2 * ch if opens == "convtranspose" else prev
        assert shapes[key + ".w1"] == (ch, cin, k, k), name
        assert shapes[key + ".w2"] == (ch, ch, k, k), name
        assert shapes[key + ".b1"] == (ch,) and shapes[key + ".b2"] == (ch,)
        prev = ch
    assert prev == 1
    # nothing beyond the table's layers
    used = {n.split(".")[0] for n in shapes}
    assert used == {"inc", "outc"} | {f"down{i}" for i in range(1, depth + 1)} | {f"up{i}" for i in range(depth)}
